// ara_kernels.hip -- gfx950 kernels of libara.
//
// Layout of the work (Algorithm 1 of Varghese & Rau-Chaplin, section 2.2):
//   * one 64-lane wavefront per trial; the trial's event ids stream from HBM
//     64 at a time (one coalesced 256-byte row per wave per chunk);
//   * each event id gathers one 16-byte row of the layer table (which XELTs
//     hold the event, where their entries sit) -- the tables are built per
//     run in event-major order so one row replaces J direct-table probes;
//   * the (event, XELT) hits of a chunk are compacted into an LDS queue with a
//     wave prefix sum and drained 64 draws at a time, so the variable-cost
//     inverse Beta runs on full waves rather than on one thread per trial;
//   * per-event sums are formed in XELT order, the occurrence terms applied
//     per event, and the trial's cumulative loss is a compensated (Neumaier)
//     per-lane sum combined across lanes with TwoSum in a fixed butterfly, so
//     every YLT value is a deterministic function of its trial.
#include "ara_internal.hpp"
#include "ara_wave.hpp"

namespace ara {

// ===========================================================================
// Load-time kernels
// ===========================================================================
__global__ void k_elt_index(const int32_t* __restrict__ event_id, int32_t n, int32_t* __restrict__ idx)
{
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) idx[event_id[r]] = r;
}

// Section 3.3 moment matching, per entry, in FP64.
__global__ void k_elt_prepare(int32_t n, const double* __restrict__ mean, const double* __restrict__ sig_i,
                              const double* __restrict__ sig_c, const double* __restrict__ maxl,
                              EntryRec* __restrict__ ent, float2* __restrict__ cw)
{
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const double mu = mean[r], si = sig_i[r], sc = sig_c ? sig_c[r] : 0.0, mx = maxl[r];
    const double s = si + sc;                                   // sigma = sigma_I + sigma_C
    EntryRec E;
    E.maxl = (float)mx;
    if (s == 0.0) {
        E.a = 0.0; E.b = 0.0; E.lnB = mu; E.us = 0.0f;
    } else {
        const double mub = mu / mx;                             // mu_beta
        const double sbmax = sqrt(mub * (1.0 - mub));           // sigma_beta_max
        const double sb = fmin(s / mx, kSigmaClamp * sbmax);
        const double nu = (sbmax / sb) * (sbmax / sb) - 1.0;
        E.a = mub * nu;
        E.b = (1.0 - mub) * nu;
        E.lnB = log_beta(E.a, E.b);
        const double ts = (E.a + 1.0) / (E.a + E.b + 2.0);
        E.us = (float)beta_inc_lower(ts, E.a, E.b, E.lnB);
    }
    ent[r] = E;
    if (cw) {
        float2 w;
        if (sc == 0.0) w = make_float2(1.0f, 0.0f);
        else if (si == 0.0) w = make_float2(0.0f, 1.0f);
        else {
            const double wi = si / s, wc = sc / s, nrm = sqrt(wi * wi + wc * wc);
            w = make_float2((float)(wi / nrm), (float)(wc / nrm));
        }
        cw[r] = w;
    }
}

// Solve records with their start tables, one thread per entry, FP64.
__global__ void k_elt_solve(int32_t n, const EntryRec* __restrict__ ent, SolveRec* __restrict__ sol)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    sol[r] = make_solve_rec(ent[r]);
}

// Tabulated-inverse records, one thread per entry, FP64.
__global__ void k_elt_tab(int32_t n, const EntryRec* __restrict__ ent, TabRec* __restrict__ tab)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    tab[r] = make_tab_rec(ent[r]);
}

__global__ void k_validate_ids(const int32_t* __restrict__ ev, int64_t n, int32_t C, unsigned int* bad)
{
    unsigned int local = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e = ev[i];
        local += (e < 0 || e >= C) ? 1u : 0u;
    }
    if (local) atomicAdd(bad, local);
}

// ===========================================================================
// Per-run layer tables
// ===========================================================================
__global__ void k_layer_count(int32_t C, int32_t J, const EltDev* __restrict__ elts, uint4* __restrict__ rows,
                              uint32_t* __restrict__ cnt)
{
    const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= C) return;
    uint64_t mask = 0;
    for (int j = 0; j < J; ++j)
        if (elts[j].idx[e] >= 0) mask |= (uint64_t)1 << j;
    const uint32_t c = (uint32_t)__popcll(mask);
    rows[e] = make_uint4((uint32_t)mask, (uint32_t)(mask >> 32), 0u, c);
    cnt[e] = c;
}

__global__ void k_layer_fill(int32_t C, int32_t J, const EltDev* __restrict__ elts, const uint32_t* __restrict__ off,
                             uint4* __restrict__ rows, EntryRec* __restrict__ pent, float2* __restrict__ pcw,
                             SolveRec* __restrict__ psol, TermThr* __restrict__ pthr, TabRec* __restrict__ ptab)
{
    const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= C) return;
    uint4 r = rows[e];
    uint32_t o = off[e];
    r.z = o;
    uint64_t mask = (uint64_t)r.x | ((uint64_t)r.y << 32);
    uint32_t pol = 0;
    for (int rank = 0; mask; ++rank) {
        const int j = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        const EltDev& X = elts[j];
        const int32_t i = X.idx[e];
        const EntryRec E = X.ent[i];
        pent[o] = E;
        if (pcw) pcw[o] = X.cw ? X.cw[i] : make_float2(1.0f, 0.0f);
        if (psol) psol[o] = X.solve[i];
        if (pthr) pthr[o] = term_thresholds(E, X.ded, X.lim);
        if (ptab) ptab[o] = X.tab[i];
        if (rank < kRowPolBits && is_small_shape(E)) pol |= 1u << rank;
        ++o;
    }
    r.w |= pol << 7;
    rows[e] = r;
}

// Mean mode (primary uncertainty only): the loss of an event occurrence does
// not depend on the trial, so its net-of-terms occurrence loss is tabulated.
// Hashed layer table: the compact alternative to the direct table over the
// catalog (section 4.1 weighs direct access against compact layouts).  Every
// event some XELT of the layer holds gets a slot with its id and its row; the
// slot a given event lands in may vary from build to build, the rows a lookup
// returns do not.
__global__ void k_hash_clear(uint4* __restrict__ slots, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        slots[2u * i] = make_uint4(0xFFFFFFFFu, 0u, 0u, 0u);
        slots[2u * i + 1u] = make_uint4(0u, 0u, 0u, 0u);
    }
}

__global__ void k_hash_insert(int32_t C, const uint4* __restrict__ rows, uint4* __restrict__ slots, uint32_t hbits)
{
    const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= C) return;
    const uint4 r = rows[e];
    if ((r.x | r.y) == 0u) return;
    const uint32_t m = (1u << hbits) - 1u;
    for (uint32_t h = layer_hash(e, hbits);; h = (h + 1u) & m) {
        // claim the slot's key word; the rest of the slot is written by its owner alone
        if (atomicCAS((int32_t*)&slots[2u * h].x, -1, e) == -1) {
            uint4* S = slots + 2u * h;
            S[0].y = r.x;
            S[0].z = r.y;
            S[0].w = r.z;
            S[1] = make_uint4(r.w, 0u, 0u, 0u);
            return;
        }
    }
}

__global__ void k_mean_table(int32_t C, int32_t J, const EltDev* __restrict__ elts, double occR, double occL,
                             float* __restrict__ occ_tab)
{
    const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= C) return;
    double c = 0.0;
    for (int j = 0; j < J; ++j) {
        const EltDev& X = elts[j];
        const int32_t i = X.idx[e];
        if (i < 0) continue;
        const double l = X.mean[i];
        c += X.share * fmin(fmax(l - X.ded, 0.0), X.lim);
    }
    occ_tab[e] = (float)fmin(fmax(c - occR, 0.0), occL);
}

// ---- exclusive scan of uint32 counts (three passes) ----
constexpr int kScanTile = 1024;      // elements per block, 256 threads x 4

__device__ uint32_t block_excl_scan_256(uint32_t v, uint32_t* sh, uint32_t& total)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        const uint32_t o = t >= d ? sh[t - d] : 0u;
        __syncthreads();
        sh[t] += o;
        __syncthreads();
    }
    total = sh[255];
    const uint32_t incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ void k_scan_tiles(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, int64_t n,
                             uint32_t* __restrict__ tile_sums)
{
    __shared__ uint32_t sh[256];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 4;
    uint32_t v[4];
    uint32_t s = 0;
    for (int i = 0; i < 4; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0u;
        s += v[i];
    }
    uint32_t total;
    uint32_t run = block_excl_scan_256(s, sh, total);
    for (int i = 0; i < 4; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void k_scan_sums(uint32_t* __restrict__ tile_sums, int64_t n_tiles)
{
    __shared__ uint32_t sh[256];
    uint32_t carry = 0;
    for (int64_t base = 0; base < n_tiles; base += 256) {
        const int64_t i = base + threadIdx.x;
        const uint32_t v = i < n_tiles ? tile_sums[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_excl_scan_256(v, sh, total);
        if (i < n_tiles) tile_sums[i] = carry + ex;
        carry += total;
    }
}

__global__ void k_scan_add(uint32_t* __restrict__ out, int64_t n, const uint32_t* __restrict__ tile_sums)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += tile_sums[i / kScanTile];
}

// ===========================================================================
// The layer kernels
// ===========================================================================
constexpr int kChunk = 64;                   // event slots per compaction round
constexpr int kRound = 6;                    // draws per slot per drain round (7.2 KB of LDS per wavefront)
constexpr int kQueue = kChunk * kRound;      // queue capacity per wave

// The solve of a deferred draw (a small shape: the series form for its small
// side, or a degenerate entry), out of line: a call whose registers stay out
// of the layer kernel's allocation (inlined, they force spills in the
// kernel's hot loops).
__device__ __attribute__((noinline)) float deferred_loss(double z, EntryRec E, const SolveRec* R)
{
    if (E.a == 0.0) return (float)E.lnB;       // degenerate: the mean loss
    return E.maxl * inv_beta32_any(z, E, *R);
}

// The correlated draw's z (two uniforms, two FP64 normal quantiles, one
// normal CDF), out of line for the same reason.
// The event's correlated uniform u_C (one per trial and slot, the same for
// every program and XELT) and its normal quantile, formed once per event.
struct CorrEvent {
    double qc;      // Phi^-1(u_C)
    float uc;       // u_C
};
__device__ __attribute__((noinline)) CorrEvent corr_event(uint32_t trial, uint32_t slot, uint32_t seed)
{
    CorrEvent c;
    c.uc = u01(philox_word0(trial, slot, 0xFFFFFFFFu, 1u, seed, 0xFFFFFFFFu));
    c.qc = normal_quantile((double)c.uc);
    return c;
}

// One draw's z from its own uniform and the event's shared part: the same
// value draw_z<true> forms, with u_C and its quantile taken from corr_event.
__device__ __attribute__((noinline)) double corr_z(uint32_t trial, uint32_t slot, uint32_t j, uint32_t seed,
                                                   uint32_t prog, const float2* pcw, uint32_t pi, float uc, double qc)
{
    const double ui = (double)u01(philox_word0(trial, slot, j, 0u, seed, prog));
    const float2 w = pcw[pi];
    if (w.y == 0.0f) return ui;
    if (w.x == 0.0f) return (double)uc;
    return normcdf((double)w.x * normal_quantile(ui) + (double)w.y * qc);
}

// Plain path, one wave per trial.  Each chunk of 64 event slots is drained in
// rounds: the queued draws of a round are classified by cost.  Draws whose
// smaller shape parameter is at least kSmallShape take the FP32 solve alone
// and are drained 64 at a time at once.  The rest (small shapes, whose small
// side takes the series form of the solve, and degenerate entries) are few --
// a handful per chunk -- so they go to a per-wave deferred queue that is
// drained only in full waves of 64 (and once, partially, at the end of the
// trial), where the two forms do not split a solve wave.  An event whose draws
// are still deferred keeps its partial loss in a small ring of pending chunks
// and takes its occurrence terms once the last of them lands.  Every sum is a
// fixed function of the trial, so the result does not depend on the launch.
// Five wavefronts per SIMD (96 VGPRs, a few spilled; LDS allows five and a
// half): four ran 10% slower, six (80 VGPRs) spill more than they gain.
constexpr int kDefer = 128;                  // deferred-draw ring per wave (power of two)
constexpr int kRing = 4;                     // chunks that may wait for deferred draws (four register sums)
constexpr int kFinal = 0x7FFF;               // pending count of a finished (or empty) slot
constexpr float kDeferred = -1.0f;           // queue value of a deferred draw (losses are >= 0)
constexpr int kRemDefer = 24;                // an FP32 list this short joins the deferred ring

template <bool HAS_CORR, int WPB, bool TAB>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(WPB == 8 ? 3 : 5))) void k_layer_plain(YetDev y, int64_t t0, int64_t t1,
                                                          const LayerDev* __restrict__ layers, int32_t n_layers)
{
    __shared__ uint32_t qidx[WPB][kQueue];
    __shared__ uint16_t qmeta[WPB][kQueue];
    __shared__ float qv[WPB][kQueue];
    __shared__ uint16_t lst[WPB][kQueue];
    __shared__ uint32_t didx[WPB][kDefer];
    __shared__ uint32_t dmeta[WPB][kDefer];
    __shared__ double dz[HAS_CORR ? WPB : 1][HAS_CORR ? kDefer : 1];
    __shared__ double qcs[HAS_CORR ? WPB : 1][HAS_CORR ? 64 : 1];     // correlated layers: per slot Phi^-1(u_C)
    __shared__ float ucs[HAS_CORR ? WPB : 1][HAS_CORR ? 64 : 1];      //   and u_C
    __shared__ float pcs[WPB][kRing][64];
    __shared__ short pns[WPB][kRing][64];
    __shared__ int rchunk[WPB][kRing];
    __shared__ int tags[WPB][64];
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    const int64_t trial = t0 + (int64_t)blockIdx.x * WPB + w;
    if (trial >= t1) return;
    uint32_t* QI = qidx[w];          // packed entry index
    uint16_t* QM = qmeta[w];         // slot within chunk | XELT position << 8
    float* QV = qv[w];               // the draw's net loss, or kDeferred
    uint16_t* L32 = lst[w];
    uint32_t* DI = didx[w];          // deferred draws: packed entry index
    uint32_t* DM = dmeta[w];         //   slot within the trial | XELT position << 24
    double* DZ = dz[HAS_CORR ? w : 0];  //   z (correlated layers: formed in the classify pass)
    double* QC = qcs[HAS_CORR ? w : 0]; // correlated layers, per slot of the chunk: Phi^-1(u_C)
    float* UC = ucs[HAS_CORR ? w : 0];  //   and u_C
    float (*PC)[64] = pcs[w];        // pending chunks: partial event loss per slot
    short (*PN)[64] = pns[w];        //   deferred draws outstanding per slot
    int* RC = rchunk[w];             //   chunk held by each ring slot (-1: free)
    int* TG = tags[w];               // flush: the queue position handed over next, per owner lane
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    int64_t row;
    int32_t len;
    trial_range(y, trial, row, len);
    const uint32_t tr = (uint32_t)trial;

    for (int32_t l = 0; l < n_layers; ++l) {
        const LayerDev& L = layers[l];
        float S = 0.0f, Sc = 0.0f, omax = 0.0f;
        int dh = 0, dn = 0;                        // deferred ring: head, count (wave-uniform)
        if (lane < kRing) RC[lane] = -1;
        // Direct tables: each chunk's event ids are loaded one chunk ahead, so
        // a chunk waits for one load (its rows) instead of two in a chain.
        const bool direct = L.hbits == 0u;
        int32_t ev_next = 0;                       // this lane's event id in the next chunk
        if (direct && lane < len) ev_next = y.ev[row + lane];
        wave_sync();

        // Occurrence terms of every settled slot of ring slot r (its chunk's
        // rounds are over): those with no deferred draw outstanding.
        auto settle = [&](int r) {
            const int ci = RC[r];
            if (ci < 0) return;
            if (PN[r][lane] == 0) {
                const float o = xl(PC[r][lane], L.occR, L.occL);
                omax = fmaxf(omax, o);
                neumaier_add(S, Sc, o);
                if (L.yelt) L.yelt[row + ci * kChunk + lane - L.yelt_base] = o;
                PN[r][lane] = kFinal;
            }
            const bool settled = __ballot(PN[r][lane] != kFinal) == 0ull;
            wave_sync();                 // every lane has read RC[r]
            if (settled && lane == 0) RC[r] = -1;
            wave_sync();
        };
        // Evaluate the m <= 64 oldest deferred draws, one per lane, then add
        // each value to the partial loss of its event slot's ring entry.
        auto flush = [&](int m, int open_ring) {
            const int e = (dh + lane) & (kDefer - 1);
            float v = 0.0f;
            uint32_t key = 0;
            if (lane < m) {
                const uint32_t pi = DI[e], meta = DM[e];
                const uint32_t j = meta >> 24;
                key = meta & 0xFFFFFFu;
                const EntryRec E = L.pent[pi];
                const double z = HAS_CORR ? DZ[e] : draw_z<false>(tr, key, j, L.seed, L.prog, nullptr, pi);
                const float loss = deferred_loss(z, E, L.psol + pi);
                const float4 jt = L.jt[j];
                v = jt.z * xl(loss, jt.x, jt.y);
            }
            // each value goes to its event slot's partial loss in rounds: per
            // round one value per owner lane, the pending one latest in the queue
            // (an LDS max over the lanes), so no two adds of a round meet; an
            // owner with k values in the flush takes k rounds (most take one)
            const uint32_t own_i = key & 63u, rs_i = (key >> 6) & (uint32_t)(kRing - 1);
            bool pend = lane < m;
            while (__ballot(pend) != 0ull) {
                if (pend) TG[own_i] = -1;
                wave_sync();
                if (pend) atomicMax(&TG[own_i], lane);
                wave_sync();
                const bool win = pend && TG[own_i] == lane;
                if (win) {
                    PC[rs_i][own_i] += v;
                    PN[rs_i][own_i] -= 1;
                }
                wave_sync();
                pend = pend && !win;
            }
            dh = __builtin_amdgcn_readfirstlane((dh + m) & (kDefer - 1));
            dn = __builtin_amdgcn_readfirstlane(dn - m);
            wave_sync();
            for (int r = 0; r < kRing; ++r)
                if (r != open_ring) settle(r);
        };

        for (int32_t ci = 0;; ++ci) {
            const int32_t base = ci * kChunk;
            const bool more = base < len;
            const int r = ci & (kRing - 1);
            // the ring slot must be free, and nothing may stay deferred past the trial
            if (!more || RC[r] >= 0)
                while (dn > 0) flush(dn < 64 ? dn : 64, -1);
            if (!more) break;
            wave_sync();                     // every lane has read RC[r] before lane 0 rewrites it
            PC[r][lane] = 0.0f;
            PN[r][lane] = 0;
            if (lane == 0) RC[r] = ci;
            wave_sync();

            const int32_t k = base + lane;
            const bool valid = k < len;
            uint4 rr = make_uint4(0, 0, 0, 0);
            if (direct) {
                if (valid) rr = L.rows[ev_next];
                if (k + kChunk < len) ev_next = y.ev[row + k + kChunk];
            } else if (valid) {
                rr = layer_row(L, y.ev[row + k]);
            }
            if (HAS_CORR) {
                // the event's correlated uniform and its quantile, once per slot
                CorrEvent ce{0.0, 0.0f};
                if (valid && (rr.x | rr.y) != 0u) ce = corr_event(tr, (uint32_t)k, L.seed);
                QC[lane] = ce.qc;
                UC[lane] = ce.uc;
            }
            uint64_t mask = (uint64_t)rr.x | ((uint64_t)rr.y << 32);
            const uint32_t off = rr.z;
            const uint32_t rw = rr.w;
            int remaining = row_count(rw);
            int rank = 0;
            bool first_round = true;         // wave-uniform
            float c = 0.0f;                  // this event's loss across XELTs, deferred draws aside
            int pend = 0;                    // its deferred draws
            while (true) {
                const int take = remaining < kRound ? remaining : kRound;
                const int incl = wave_incl_scan(take);
                const int total = __builtin_amdgcn_readlane(incl, 63);     // wave-uniform (scalar)
                if (total == 0) break;
                const int pos = incl - take;
                for (int i = 0; i < take; ++i) {
                    const int j = __ffsll((unsigned long long)mask) - 1;
                    mask &= mask - 1;
                    const int rk = rank + i;
                    // the table mode takes every draw from its table: nothing is deferred
                    const uint32_t pol = TAB ? 0u : rk < kRowPolBits ? (rw >> (7 + rk)) & 1u : L.psol[off + (uint32_t)rk].pol;
                    QI[pos + i] = off + (uint32_t)rk;
                    QM[pos + i] = (uint16_t)(lane | (pol << 7) | (j << 8));
                }
                wave_sync();
                // (A) classify: draws whose term the quantile cannot change take
                // it here; the other FP32 draws go to the list, the rest to the
                // deferred ring
                int n32 = 0;
                for (int b0 = 0; b0 < total; b0 += 64) {
                    const int q = b0 + lane;
                    const bool in = q < total;
                    bool pol = false, keep = in;
                    // the draw's z is formed here, once per draw in full waves, and
                    // kept for the solve (correlated layers: two uniforms and the
                    // normal transforms in FP64)
                    double zc = 0.0;
                    if (in) {
                        const uint32_t pi = QI[q], meta = QM[q];
                        const uint32_t own = meta & 63u, j = meta >> 8;
                        pol = (meta & 0x80u) != 0u;
                        zc = HAS_CORR ? corr_z(tr, (uint32_t)base + own, j, L.seed, L.prog, L.pcw, pi, UC[own], QC[own])
                                      : draw_z<false>(tr, (uint32_t)base + own, j, L.seed, L.prog, nullptr, pi);
                        // the loss would lie within the retention, or beyond retention +
                        // limit (term_thresholds): the term is 0 or the limit, no solve
                        const TermThr th = L.pthr[pi];
                        if (zc <= (double)thr_lo(th)) {
                            QV[q] = 0.0f;
                            keep = false;
                        } else if (zc >= (double)thr_hi(th)) {
                            const float4 jt = L.jt[j];
                            QV[q] = jt.z * jt.y;
                            keep = false;
                        }
                    }
                    const uint64_t b64 = __ballot(keep && pol);
                    const uint64_t b32 = __ballot(keep && !pol);
                    if (keep) {
                        if (pol) {
                            const int e = (dh + dn + __popcll(b64 & below)) & (kDefer - 1);
                            const uint32_t meta = QM[q];
                            DI[e] = QI[q];
                            DM[e] = ((uint32_t)base + (meta & 63u)) | ((meta >> 8) << 24);
                            if (HAS_CORR) DZ[e] = zc;
                            QV[q] = kDeferred;
                        } else {
                            L32[n32 + __popcll(b32 & below)] = (uint16_t)q;
                            // the FP32 solve takes z as its tail code (uncorrelated draws are
                            // on the 2^-24 grid, where the code is z itself, exactly)
                            QV[q] = HAS_CORR ? tail_code(zc) : (float)zc;
                        }
                    }
                    n32 = __builtin_amdgcn_readfirstlane(n32 + __popcll(b32));
                    dn = __builtin_amdgcn_readfirstlane(dn + __popcll(b64));
                    wave_sync();
                    if (dn >= 64) flush(64, r);
                }
                // A chunk whose first round's FP32 list is short (sparse layers: a
                // few draws per chunk) sends it to the deferred ring, which solves
                // in full waves across chunks, instead of solving a nearly empty
                // wave here.  In dense chunks, and in the short later rounds of
                // events with many hits, the ring costs more than the partial wave
                // it would save.  (Correlated layers keep it: the ring would need
                // each draw's z in FP64.)
                if (!HAS_CORR && !TAB && first_round && n32 != 0 && n32 <= kRemDefer) {
                    const int rem = n32, n0 = 0;
                    if (lane < rem) {
                        const int q = L32[n0 + lane];
                        const uint32_t meta = QM[q];
                        const int e = (dh + dn + lane) & (kDefer - 1);
                        DI[e] = QI[q];
                        DM[e] = ((uint32_t)base + (meta & 63u)) | ((meta >> 8) << 24);
                        QV[q] = kDeferred;
                    }
                    dn = __builtin_amdgcn_readfirstlane(dn + rem);
                    n32 = n0;
                    wave_sync();
                    if (dn >= 64) flush(64, r);
                }
                // (B) FP32 solve
                for (int b0 = 0; b0 < n32; b0 += 64) {
                    const int idx = b0 + lane;
                    if (idx < n32) {
                        const int q = L32[idx];
                        const uint32_t pi = QI[q], j = QM[q] >> 8;
                        // the draw's z from the classify pass (uncorrelated draws are on the
                        // 2^-24 grid; correlated ones arrive as tail codes)
                        const float z = QV[q];
                        float loss;
                        if (TAB) {
                            const TabRec& T = L.ptab[pi];
                            loss = T.maxl * (HAS_CORR ? tab_inverse_code(z, T) : tab_inverse(z, T));
                        } else {
                            const SolveRec& R = L.psol[pi];
                            loss = R.maxl * (HAS_CORR ? inv_beta32_code(z, R) : inv_beta32(z, R));
                        }
                        const float4 jt = L.jt[j];
                        QV[q] = jt.z * xl(loss, jt.x, jt.y);                  // per-XELT terms
                    }
                }
                wave_sync();
                for (int i = 0; i < take; ++i) {
                    const float v = QV[pos + i];
                    if (v == kDeferred) ++pend;
                    else c += v;
                }
                rank += take;
                remaining -= take;
                first_round = false;
                wave_sync();
            }
            // the chunk's rounds are over: slots with nothing deferred settle now
            PC[r][lane] += c;
            PN[r][lane] = valid ? PN[r][lane] + pend : kFinal;
            wave_sync();
            settle(r);
        }
        wave_sum_pair(S, Sc);
        omax = wave_max(omax);
        if (lane == 0) {
            const float Y = fminf(fmaxf((S - L.aggR) + Sc, 0.0f), L.aggL);   // aggregate terms
            L.ylt[trial - t0] = Y;
            if (L.omax) L.omax[trial - t0] = omax;
        }
        wave_sync();
    }
}

// Mean mode (the streaming phase): the per-event loss net of XELT and
// occurrence terms is tabulated per event (k_mean_table), so a trial's year
// loss is the sum of one table value per event.  Gathering those values from
// L2 caps the rate at the L2 request rate, far below HBM.  Instead the
// catalog is cut into slices of 72 KB of LDS (two workgroups of 16
// wavefronts fill a CU's 160 KB and its 32 wavefront slots), and the YET
// gets a slice-major copy (once per YET, k_yet_slice): each trial's ids
// regrouped by slice, each group padded with -1 to a multiple of four.
// Workgroup (tile, slice) holds its slice of the table in LDS and streams
// only that slice's ids of its trials, so every id is read once.
// k_mean_finish adds a trial's slice sums in slice order (FP64) and applies
// the aggregate terms.  Catalogs of more than kMaxSlices slices use
// k_mean_gather, which reads the table through L2.
constexpr int kSliceMax = 18432;             // table entries per slice (72 KB of LDS: two workgroups per CU)
constexpr int kMaxSlices = 16;
constexpr int kMeanWaves = 16;               // wavefronts per workgroup
constexpr int kMeanTile = 1024;              // trials per workgroup
constexpr int kLanesPerTrial = 8;            // lanes streaming one trial's group
constexpr int kTrialsPerWave = 64 / kLanesPerTrial;
constexpr int kMeanPre = 3;                 // 16-byte loads per lane kept in flight one batch ahead
constexpr int kGroupAlign = 8;              // ids per 16-byte load of the slice-major copy
constexpr uint16_t kSlicePad = 0xFFFF;      // padding id (beyond every slice)

// The slice-major copy: group (slice s, trial t) holds trial t's ids that
// fall in slice s, in time order, as 16-bit offsets into the slice (a slice
// has at most kSliceMax < 2^16 events), padded with kSlicePad to a multiple
// of eight (one 16-byte load); the groups of one slice are consecutive over
// the trials, slice after slice, so a workgroup streams one contiguous run.
// k_yet_count sizes the groups, an exclusive scan over (slice, trial) places
// them, k_yet_scatter fills them.
__global__ __launch_bounds__(256) void k_yet_count(YetDev y, int32_t slice_len, int32_t ns, uint32_t* __restrict__ cnt)
{
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= y.N) return;
    const int lane = lane_id();
    int64_t row;
    int32_t len;
    trial_range(y, t, row, len);
    for (int32_t sl = 0; sl < ns; ++sl) {
        int32_t c = 0;
        for (int32_t k0 = 0; k0 < len; k0 += 64) {
            const int32_t k = k0 + lane;
            c += __popcll(__ballot(k < len && y.ev[row + k] / slice_len == sl));
        }
        if (lane == 0) cnt[(int64_t)sl * y.N + t] = (uint32_t)((c + kGroupAlign - 1) & ~(kGroupAlign - 1));
    }
}

__global__ __launch_bounds__(256) void k_yet_scatter(YetDev y, int32_t slice_len, int32_t ns,
                                                     const uint32_t* __restrict__ off, const uint32_t* __restrict__ cnt,
                                                     uint16_t* __restrict__ ev2)
{
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= y.N) return;
    const int lane = lane_id();
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t row;
    int32_t len;
    trial_range(y, t, row, len);
    for (int32_t sl = 0; sl < ns; ++sl) {
        const int64_t g = (int64_t)sl * y.N + t;
        const int64_t start = off[g];
        int32_t fill = 0;
        for (int32_t k0 = 0; k0 < len; k0 += 64) {
            const int32_t k = k0 + lane;
            const int32_t id = k < len ? y.ev[row + k] : 0;
            const bool mine = k < len && id / slice_len == sl;
            const uint64_t m = __ballot(mine);
            if (mine) ev2[start + fill + __popcll(m & below)] = (uint16_t)(id - sl * slice_len);
            fill += __popcll(m);
        }
        for (int32_t q = fill + lane; q < (int32_t)cnt[g]; q += 64) ev2[start + q] = kSlicePad;
    }
}

// kLanesPerTrial lanes per trial, kTrialsPerWave trials per wavefront at a
// time, so each wavefront keeps several 16-byte loads of several trials in
// flight; the next batch's ids and the offsets of the batch after it are
// fetched while a batch is summed.
__global__ __launch_bounds__(64 * kMeanWaves) void k_mean_slice(YetDev y, int64_t t0, int64_t t1,
                                                                 const LayerDev* __restrict__ layers, int32_t l,
                                                                 const uint16_t* __restrict__ ev2,
                                                                 const uint32_t* __restrict__ goff,
                                                                 const uint32_t* __restrict__ gcnt, int32_t slice_len,
                                                                 int32_t ns, float2* __restrict__ part,
                                                                 float* __restrict__ pmax)
{
    __shared__ float4 stab4[kSliceMax / 4];
    const float* stab = reinterpret_cast<const float*>(stab4);
    const int64_t tile = blockIdx.x / ns;
    const int32_t sl = (int32_t)(blockIdx.x % ns);
    const LayerDev& L = layers[l];
    const int32_t lo = sl * slice_len;                   // slice_len is a multiple of 4
    const int32_t n = min(slice_len, y.C - lo);
    const float4* src4 = reinterpret_cast<const float4*>(L.occ_tab + lo);
    for (int i = threadIdx.x; i < (n >> 2); i += blockDim.x) stab4[i] = src4[i];
    for (int i = (n & ~3) + threadIdx.x; i < n; i += blockDim.x) reinterpret_cast<float*>(stab4)[i] = L.occ_tab[lo + i];
    __syncthreads();
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    const int grp = lane / kLanesPerTrial, sub = lane % kLanesPerTrial;
    const uint32_t un = (uint32_t)n;
    const int64_t nt = t1 - t0;
    const int64_t tb = tile * kMeanTile;
    const int64_t te = min(nt, tb + (int64_t)kMeanTile);
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));      // eight 16-bit ids
    // where trial i's group for this slice lives: offset into the copy, length in 16-byte loads
    auto locate = [&](int64_t i, int64_t& at, int32_t& n4) {
        at = 0;
        n4 = 0;
        if (i < te) {
            const int64_t g = (int64_t)sl * y.N + t0 + i;
            at = goff[g];
            n4 = (int32_t)(gcnt[g] / kGroupAlign);
        }
    };
    // The first kMeanPre 16-byte loads of each lane's share of a group are
    // issued one batch of trials ahead, so the next trials' ids stream in
    // while this batch is summed; a group longer than kMeanPre x kLanesPerTrial
    // loads (192 ids of one slice in one trial) reads the rest in place.
    auto fetch = [&](int64_t at_, int32_t n4_, v4u* dst) {
        const v4u* __restrict__ p = reinterpret_cast<const v4u*>(ev2 + at_);
#pragma unroll
        for (int r = 0; r < kMeanPre; ++r) {
            const int32_t q = sub + r * kLanesPerTrial;
            dst[r] = q < n4_ ? __builtin_nontemporal_load(p + q) : v4u{0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
        }
    };
    constexpr int64_t kStride = kTrialsPerWave * kMeanWaves;
    const int64_t first = tb + kTrialsPerWave * w + grp;
    int64_t at, at1;
    int32_t n4, n41;
    locate(first, at, n4);
    v4u e[kMeanPre];
    fetch(at, n4, e);
    locate(first + kStride, at1, n41);                   // offsets of the next batch
    for (int64_t i0 = tb + kTrialsPerWave * w; i0 < te; i0 += kStride) {
        const int64_t i = i0 + grp;
        const bool live = i < te;
        v4u en[kMeanPre];
        fetch(at1, n41, en);                             // the next batch's ids, in flight during this one
        int64_t at2;
        int32_t n42;
        locate(i + 2 * kStride, at2, n42);               // and the offsets of the batch after it
        float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f, m = 0.0f;
        auto add8 = [&](const v4u& x) {
            // two ids per word; the padding id is beyond every slice
            const uint32_t u0 = x.x & 0xFFFFu, u1 = x.x >> 16, u2 = x.y & 0xFFFFu, u3 = x.y >> 16;
            const uint32_t u4 = x.z & 0xFFFFu, u5 = x.z >> 16, u6 = x.w & 0xFFFFu, u7 = x.w >> 16;
            const float v0 = u0 < un ? stab[u0] : 0.0f;
            const float v1 = u1 < un ? stab[u1] : 0.0f;
            const float v2 = u2 < un ? stab[u2] : 0.0f;
            const float v3 = u3 < un ? stab[u3] : 0.0f;
            const float v4 = u4 < un ? stab[u4] : 0.0f;
            const float v5 = u5 < un ? stab[u5] : 0.0f;
            const float v6 = u6 < un ? stab[u6] : 0.0f;
            const float v7 = u7 < un ? stab[u7] : 0.0f;
            a0 += v0 + v4;
            a1 += v1 + v5;
            a2 += v2 + v6;
            a3 += v3 + v7;
            m = fmaxf(m, fmaxf(fmaxf(fmaxf(v0, v1), fmaxf(v2, v3)), fmaxf(fmaxf(v4, v5), fmaxf(v6, v7))));
        };
#pragma unroll
        for (int r = 0; r < kMeanPre; ++r) add8(e[r]);
        const v4u* __restrict__ v8 = reinterpret_cast<const v4u*>(ev2 + at);
#pragma unroll 1
        for (int32_t q = sub + kMeanPre * kLanesPerTrial; q < n4; q += kLanesPerTrial)
            add8(__builtin_nontemporal_load(v8 + q));
#pragma unroll
        for (int r = 0; r < kMeanPre; ++r) e[r] = en[r];
        at = at1;
        n4 = n41;
        at1 = at2;
        n41 = n42;
        float S = a0, Sc = 0.0f;
        neumaier_add(S, Sc, a1);
        neumaier_add(S, Sc, a2);
        neumaier_add(S, Sc, a3);
#pragma unroll
        for (int k = kLanesPerTrial / 2; k >= 1; k >>= 1) {   // within the trial's lanes
            const float oh = __shfl_xor(S, k, kLanesPerTrial);
            const float ol = __shfl_xor(Sc, k, kLanesPerTrial);
            two_sum_merge(S, Sc, oh, ol);
            m = fmaxf(m, __shfl_xor(m, k, kLanesPerTrial));
        }
        if (live && sub == 0) {
            part[(int64_t)sl * nt + i] = make_float2(S, Sc);
            if (L.omax) pmax[(int64_t)sl * nt + i] = m;      // only when the largest occurrence is asked for
        }
    }
}

__global__ __launch_bounds__(256) void k_mean_finish(const LayerDev* __restrict__ layers, int32_t l, int64_t nt,
                                                     int32_t ns, const float2* __restrict__ part,
                                                     const float* __restrict__ pmax)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt) return;
    const LayerDev& L = layers[l];
    double S = 0.0;
    float m = 0.0f;
    for (int32_t sl = 0; sl < ns; ++sl) {
        const float2 p = part[(int64_t)sl * nt + i];
        S += (double)p.x + (double)p.y;
        if (L.omax) m = fmaxf(m, pmax[(int64_t)sl * nt + i]);
    }
    L.ylt[i] = (float)fmin(fmax(S - (double)L.aggR, 0.0), (double)L.aggL);    // aggregate terms
    if (L.omax) L.omax[i] = m;
}

// Per-occurrence output of the mean mode: each occurrence's tabulated loss,
// in the YET's layout (written beside the sums, which it does not change).
__global__ __launch_bounds__(256) void k_mean_yelt(YetDev y, int64_t t0, int64_t t1,
                                                   const LayerDev* __restrict__ layers, int32_t l)
{
    const LayerDev& L = layers[l];
    if (!L.yelt) return;
    const int64_t r0 = y.offs ? y.offs[t0] : t0 * (int64_t)y.K;
    const int64_t r1 = y.offs ? y.offs[t1] : t1 * (int64_t)y.K;
    for (int64_t r = r0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < r1;
         r += (int64_t)gridDim.x * blockDim.x)
        L.yelt[r - L.yelt_base] = L.occ_tab[y.ev[r]];
}

// Per-occurrence aggregate increments (section 2.3 applies the aggregate terms
// to the running sum of a trial's occurrence losses, so each occurrence's
// share of the year loss depends on the events before it).  With S_k the sum
// of the trial's occurrence losses up to and including occurrence k (FP64)
// and A_k = min(max(S_k - AggR, 0), AggL), occurrence k's increment is
// A_k - A_{k-1} (A_{-1} = 0); the increments of a trial add up to A of its
// last occurrence, its year loss.  One wavefront per trial, 64 occurrences
// at a time through an FP64 wave prefix sum.
__global__ __launch_bounds__(256) void k_yelt_increments(YetDev y, int64_t t0, int64_t t1, int64_t base, double aggR,
                                                         double aggL, const float* __restrict__ occ,
                                                         float* __restrict__ inc)
{
    const int lane = lane_id();
    const int64_t trial = t0 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (trial >= t1) return;
    int64_t row;
    int32_t len;
    trial_range(y, trial, row, len);
    double carry = 0.0, aprev = 0.0;          // S and A before the chunk
    for (int32_t k0 = 0; k0 < len; k0 += 64) {
        const int32_t k = k0 + lane;
        double v = k < len ? (double)occ[row + k - base] : 0.0;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const double o = __shfl_up(v, d, 64);
            if (lane >= d) v += o;
        }
        const double S = carry + v;
        const double A = fmin(fmax(S - aggR, 0.0), aggL);
        const double Ab = __shfl_up(A, 1, 64);
        if (k < len) inc[row + k - base] = (float)(A - (lane == 0 ? aprev : Ab));
        carry = __shfl(S, 63, 64);            // lanes past the trial's end add nothing
        aprev = __shfl(A, 63, 64);
    }
}

// Large catalogs: one wavefront per trial gathers the table through L2.
__global__ __launch_bounds__(256) void k_mean_gather(YetDev y, int64_t t0, int64_t t1,
                                                     const LayerDev* __restrict__ layers, int32_t n_layers)
{
    const int lane = lane_id();
    const int64_t trial = t0 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (trial >= t1) return;
    int64_t row;
    int32_t len;
    trial_range(y, trial, row, len);
    for (int32_t l = 0; l < n_layers; ++l) {
        const LayerDev& L = layers[l];
        float S = 0.0f, Sc = 0.0f, omax = 0.0f;
        for (int32_t k = lane; k < len; k += 64) {
            const float a = L.occ_tab[y.ev[row + k]];
            neumaier_add(S, Sc, a);
            omax = fmaxf(omax, a);
        }
        wave_sum_pair(S, Sc);
        omax = wave_max(omax);
        if (lane == 0) {
            L.ylt[trial - t0] = fminf(fmaxf((S - L.aggR) + Sc, 0.0f), L.aggL);
            if (L.omax) L.omax[trial - t0] = omax;
        }
    }
}

// ===========================================================================
// PML / TVaR: radix select of the k-th largest year loss (four 8-bit digits of
// an order-preserving key), then an FP64 sum of everything above it.
// ===========================================================================
__device__ __forceinline__ uint32_t order_key(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_value(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

struct KList {
    uint32_t k[kMaxRp];
};

__global__ void k_rm_init(uint32_t* state, uint32_t* hist, KList ks, int32_t n_rp)
{
    const int t = threadIdx.x;
    if (t < n_rp) {
        state[2 * t] = 0u;            // key prefix found so far
        state[2 * t + 1] = ks.k[t];   // rank still to find inside the prefix
    }
    for (int i = t; i < kMaxRp * 256; i += blockDim.x) hist[i] = 0u;
}

__global__ __launch_bounds__(256) void k_rm_hist(const float* __restrict__ y, int64_t n, int32_t n_rp, int shift,
                                                 const uint32_t* __restrict__ state, uint32_t* __restrict__ hist)
{
    __shared__ uint32_t lh[kMaxRp][256];
    for (int i = threadIdx.x; i < n_rp * 256; i += blockDim.x) lh[i >> 8][i & 255] = 0u;
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t key = order_key(y[i]);
        for (int r = 0; r < n_rp; ++r) {
            const uint32_t pre = state[2 * r];
            const bool match = (shift == 24) ? true : (((key ^ pre) >> (shift + 8)) == 0u);
            if (match) atomicAdd(&lh[r][(key >> shift) & 255u], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n_rp * 256; i += blockDim.x) {
        const uint32_t v = lh[i >> 8][i & 255];
        if (v) atomicAdd(&hist[i], v);
    }
}

__global__ void k_rm_pick(uint32_t* state, uint32_t* hist, int32_t n_rp, int shift)
{
    const int r = threadIdx.x;
    if (r < n_rp) {
        uint32_t need = state[2 * r + 1];
        uint32_t cum = 0;
        int d = 255;
        for (; d > 0; --d) {
            const uint32_t h = hist[r * 256 + d];
            if (cum + h >= need) break;
            cum += h;
        }
        state[2 * r] |= (uint32_t)d << shift;
        state[2 * r + 1] = need - cum;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kMaxRp * 256; i += blockDim.x) hist[i] = 0u;
}

__global__ __launch_bounds__(256) void k_rm_tail(const float* __restrict__ y, int64_t n, int32_t n_rp,
                                                 const uint32_t* __restrict__ state, double* __restrict__ partial)
{
    __shared__ double sh[kMaxRp][256];
    double acc[kMaxRp];
    uint32_t thr[kMaxRp];
    for (int r = 0; r < kMaxRp; ++r) {
        acc[r] = 0.0;
        thr[r] = r < n_rp ? state[2 * r] : 0xFFFFFFFFu;
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float v = y[i];
        const uint32_t key = order_key(v);
#pragma unroll
        for (int r = 0; r < kMaxRp; ++r)
            if (key > thr[r]) acc[r] += (double)v;
    }
    for (int r = 0; r < n_rp; ++r) sh[r][threadIdx.x] = acc[r];
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if ((int)threadIdx.x < d)
            for (int r = 0; r < n_rp; ++r) sh[r][threadIdx.x] += sh[r][threadIdx.x + d];
        __syncthreads();
    }
    if ((int)threadIdx.x < n_rp) partial[blockIdx.x * kMaxRp + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_rm_final(const uint32_t* __restrict__ state, const double* __restrict__ partial, int32_t nblk,
                           KList ks, int32_t n_rp, double* __restrict__ out)
{
    const int r = threadIdx.x;
    if (r >= n_rp) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[b * kMaxRp + r];
    const double v = (double)key_value(state[2 * r]);
    const double k = (double)ks.k[r];
    out[2 * r] = v;                                        // PML: the k-th largest
    out[2 * r + 1] = (s + (double)state[2 * r + 1] * v) / k; // TVaR: mean of the k largest
}

// ===========================================================================
// Auxiliary kernels: uniforms and quantiles for arbitrary inputs
// ===========================================================================
__global__ void k_philox_uniforms(const uint4* __restrict__ ctr, int64_t n, uint32_t k0, uint32_t k1,
                                  float* __restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 c = ctr[i];
    out[i] = u01(philox_word0(c.x, c.y, c.z, c.w, k0, k1));
}

__global__ void k_beta_quantile(const double* __restrict__ a, const double* __restrict__ b,
                                const double* __restrict__ u, int64_t n, double* __restrict__ x)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    EntryRec E;
    E.a = a[i];
    E.b = b[i];
    E.lnB = log_beta(E.a, E.b);
    E.us = (float)beta_inc_lower((E.a + 1.0) / (E.a + E.b + 2.0), E.a, E.b, E.lnB);
    E.maxl = 1.0f;
    x[i] = inv_beta(u[i], E);
}

__global__ void k_beta_quantile_layer(const double* __restrict__ a, const double* __restrict__ b,
                                      const double* __restrict__ u, int64_t n, double* __restrict__ x)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    EntryRec E;
    E.a = a[i];
    E.b = b[i];
    E.lnB = log_beta(E.a, E.b);
    E.us = (float)beta_inc_lower((E.a + 1.0) / (E.a + E.b + 2.0), E.a, E.b, E.lnB);
    E.maxl = 1.0f;
    const SolveRec R = make_solve_rec(E);           // as the layer tables hold it
    x[i] = inv_beta_layer(u[i], E, R);
}

// ===========================================================================
// Launchers
// ===========================================================================
__global__ void k_beta_quantile_table(const double* __restrict__ a, const double* __restrict__ b,
                                      const double* __restrict__ u, int64_t n, double* __restrict__ x)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    EntryRec E;
    E.a = a[i];
    E.b = b[i];
    E.lnB = log_beta(E.a, E.b);
    E.us = (float)beta_inc_lower((E.a + 1.0) / (E.a + E.b + 2.0), E.a, E.b, E.lnB);
    E.maxl = 1.0f;
    const TabRec T = make_tab_rec(E);               // as the table mode holds it
    x[i] = (double)tab_inverse_code(tail_code(u[i]), T);
}

hipError_t launch_beta_quantile_table(const double* a, const double* b, const double* u, int64_t n, double* x,
                                      hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_beta_quantile_table, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, a, b, u, n, x);
    return hipGetLastError();
}

hipError_t launch_beta_quantile_layer(const double* a, const double* b, const double* u, int64_t n, double* x,
                                      hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_beta_quantile_layer, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, a, b, u, n, x);
    return hipGetLastError();
}

hipError_t launch_philox_uniforms(const uint32_t* ctr, int64_t n, uint32_t k0, uint32_t k1, float* out, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_philox_uniforms, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           (const uint4*)ctr, n, k0, k1, out);
    return hipGetLastError();
}

__global__ void k_normal_quantile(const double* __restrict__ p, int64_t n, double* __restrict__ x)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = normal_quantile(p[i]);
}

hipError_t launch_normal_quantile(const double* p, int64_t n, double* x, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_normal_quantile, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, x);
    return hipGetLastError();
}

hipError_t launch_beta_quantile(const double* a, const double* b, const double* u, int64_t n, double* x, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_beta_quantile, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, a, b, u, n, x);
    return hipGetLastError();
}

static inline unsigned nblocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_elt_index(const int32_t* event_id, int32_t n, int32_t* idx, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_elt_index, dim3(nblocks(n, 256)), dim3(256), 0, s, event_id, n, idx);
    return hipGetLastError();
}

hipError_t launch_elt_prepare(int32_t n, const double* mean, const double* sig_i, const double* sig_c,
                              const double* maxl, EntryRec* ent, float2* cw, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_elt_prepare, dim3(nblocks(n, 128)), dim3(128), 0, s, n, mean, sig_i, sig_c, maxl, ent, cw);
    return hipGetLastError();
}

hipError_t launch_elt_tab(int32_t n, const EntryRec* ent, TabRec* tab, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_elt_tab, dim3(nblocks(n, 64)), dim3(64), 0, s, n, ent, tab);
    return hipGetLastError();
}

hipError_t launch_elt_solve(int32_t n, const EntryRec* ent, SolveRec* sol, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_elt_solve, dim3(nblocks(n, 64)), dim3(64), 0, s, n, ent, sol);
    return hipGetLastError();
}

hipError_t launch_validate_ids(const int32_t* ev, int64_t n, int32_t C, unsigned int* bad, hipStream_t s)
{
    if (n > 0) {
        const unsigned g = (unsigned)std::min<int64_t>(4096, (n + 255) / 256);
        hipLaunchKernelGGL(k_validate_ids, dim3(g), dim3(256), 0, s, ev, n, C, bad);
    }
    return hipGetLastError();
}

hipError_t launch_layer_count(int32_t C, int32_t J, const EltDev* elts, uint4* rows, uint32_t* cnt, hipStream_t s)
{
    hipLaunchKernelGGL(k_layer_count, dim3(nblocks(C, 256)), dim3(256), 0, s, C, J, elts, rows, cnt);
    return hipGetLastError();
}

size_t scan_scratch_words(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 1; }

hipError_t launch_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* scratch, hipStream_t s)
{
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(256), 0, s, in, out, n, scratch);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, scratch, tiles);
    hipLaunchKernelGGL(k_scan_add, dim3(nblocks(n, 256)), dim3(256), 0, s, out, n, (const uint32_t*)scratch);
    return hipGetLastError();
}

hipError_t launch_layer_fill(int32_t C, int32_t J, const EltDev* elts, const uint32_t* off, uint4* rows,
                             EntryRec* pent, float2* pcw, SolveRec* psol, TermThr* pthr, TabRec* ptab,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_layer_fill, dim3(nblocks(C, 256)), dim3(256), 0, s, C, J, elts, off, rows, pent, pcw, psol,
                       pthr, ptab);
    return hipGetLastError();
}

hipError_t launch_mean_table(int32_t C, int32_t J, const EltDev* elts, double occR, double occL, float* occ_tab,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_mean_table, dim3(nblocks(C, 256)), dim3(256), 0, s, C, J, elts, occR, occL, occ_tab);
    return hipGetLastError();
}

template <int WPB>
static void launch_layers_wpb(int mode, bool has_corr, const YetDev& y, int64_t t0, int64_t t1, const LayerDev* layers,
                              int32_t n_layers, hipStream_t s)
{
    const int64_t n = t1 - t0;
    const dim3 grid(nblocks(n, WPB)), block(64 * WPB);
    const bool tab = mode == kModeTable;
    if (has_corr && tab)
        hipLaunchKernelGGL((k_layer_plain<true, WPB, true>), grid, block, 0, s, y, t0, t1, layers, n_layers);
    else if (has_corr)
        hipLaunchKernelGGL((k_layer_plain<true, WPB, false>), grid, block, 0, s, y, t0, t1, layers, n_layers);
    else if (tab)
        hipLaunchKernelGGL((k_layer_plain<false, WPB, true>), grid, block, 0, s, y, t0, t1, layers, n_layers);
    else
        hipLaunchKernelGGL((k_layer_plain<false, WPB, false>), grid, block, 0, s, y, t0, t1, layers, n_layers);
}

int32_t mean_slices(int32_t C)
{
    const int32_t ns = (C + kSliceMax - 1) / kSliceMax;
    return ns <= kMaxSlices ? ns : 0;
}

int32_t mean_slice_len(int32_t C)
{
    const int32_t ns = mean_slices(C);
    return ns ? (((C + ns - 1) / ns + 3) & ~3) : 0;       // a multiple of 4, at most kSliceMax
}

size_t mean_workspace_bytes(int32_t C, int64_t n_trials)
{
    return (size_t)std::max<int32_t>(1, mean_slices(C)) * (size_t)n_trials * 12;
}

hipError_t launch_yet_slice_count(const YetDev& y, uint32_t* cnt, hipStream_t s)
{
    const int32_t ns = mean_slices(y.C);
    if (y.N <= 0 || ns == 0) return hipSuccess;
    hipLaunchKernelGGL(k_yet_count, dim3(nblocks(y.N, 4)), dim3(256), 0, s, y, mean_slice_len(y.C), ns, cnt);
    return hipGetLastError();
}

hipError_t launch_yet_slice_scatter(const YetDev& y, const uint32_t* off, const uint32_t* cnt, uint16_t* ev2,
                                    hipStream_t s)
{
    const int32_t ns = mean_slices(y.C);
    if (y.N <= 0 || ns == 0) return hipSuccess;
    hipLaunchKernelGGL(k_yet_scatter, dim3(nblocks(y.N, 4)), dim3(256), 0, s, y, mean_slice_len(y.C), ns, off, cnt,
                       ev2);
    return hipGetLastError();
}

hipError_t launch_mean(const YetDev& y, int64_t t0, int64_t t1, const LayerDev* layers, int32_t n_layers,
                       const uint16_t* ev2, const uint32_t* goff, const uint32_t* gcnt, void* ws, bool yelt,
                       hipStream_t s)
{
    const int64_t nt = t1 - t0;
    if (nt <= 0 || n_layers <= 0) return hipSuccess;
    if (yelt)
        for (int32_t l = 0; l < n_layers; ++l)
            hipLaunchKernelGGL(k_mean_yelt, dim3(2048), dim3(256), 0, s, y, t0, t1, layers, l);
    const int32_t ns = mean_slices(y.C);
    if (ns == 0 || !ev2) {
        hipLaunchKernelGGL(k_mean_gather, dim3(nblocks(nt, 4)), dim3(256), 0, s, y, t0, t1, layers, n_layers);
        return hipGetLastError();
    }
    const int64_t n_tiles = (nt + kMeanTile - 1) / kMeanTile;
    float2* part = (float2*)ws;
    float* pmax = (float*)((char*)ws + (size_t)ns * nt * 8);
    for (int32_t l = 0; l < n_layers; ++l) {
        hipLaunchKernelGGL(k_mean_slice, dim3((unsigned)(n_tiles * ns)), dim3(64 * kMeanWaves), 0, s, y, t0, t1,
                           layers, l, ev2, goff, gcnt, mean_slice_len(y.C), ns, part, pmax);
        hipLaunchKernelGGL(k_mean_finish, dim3(nblocks(nt, 256)), dim3(256), 0, s, layers, l, nt, ns,
                           (const float2*)part, (const float*)pmax);
    }
    return hipGetLastError();
}

hipError_t launch_layers(int mode, bool has_corr, const YetDev& y, int64_t t0, int64_t t1, const LayerDev* layers,
                         int32_t n_layers, int32_t wpb, hipStream_t s)
{
    if (t1 - t0 <= 0 || n_layers <= 0) return hipSuccess;
    switch (wpb) {
        case 1: launch_layers_wpb<1>(mode, has_corr, y, t0, t1, layers, n_layers, s); break;
        case 2: launch_layers_wpb<2>(mode, has_corr, y, t0, t1, layers, n_layers, s); break;
        case 8: launch_layers_wpb<8>(mode, has_corr, y, t0, t1, layers, n_layers, s); break;
        default: launch_layers_wpb<4>(mode, has_corr, y, t0, t1, layers, n_layers, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_yelt_increments(const YetDev& y, int64_t t0, int64_t t1, int64_t base, double aggR, double aggL,
                                  const float* occ, float* inc, hipStream_t s)
{
    if (t1 > t0)
        hipLaunchKernelGGL(k_yelt_increments, dim3(nblocks(t1 - t0, 4)), dim3(256), 0, s, y, t0, t1, base, aggR, aggL,
                           occ, inc);
    return hipGetLastError();
}

// Portfolio and program totals: per trial, the sum of n year-loss tables in
// FP64, in the order given.
__global__ __launch_bounds__(256) void k_sum_ylts(const float* const* __restrict__ ylts, int32_t n, int64_t nt,
                                                  float* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt) return;
    double s = 0.0;
    for (int32_t l = 0; l < n; ++l) s += (double)ylts[l][i];
    out[i] = (float)s;
}

hipError_t launch_sum_ylts(const float* const* ylts_dev, int32_t n, int64_t nt, float* out, hipStream_t s)
{
    if (nt > 0) hipLaunchKernelGGL(k_sum_ylts, dim3(nblocks(nt, 256)), dim3(256), 0, s, ylts_dev, n, nt, out);
    return hipGetLastError();
}

hipError_t launch_layer_hash(int32_t C, const uint4* rows, uint4* slots, uint32_t hbits, hipStream_t s)
{
    const uint32_t n = 1u << hbits;
    hipLaunchKernelGGL(k_hash_clear, dim3((n + 255) / 256), dim3(256), 0, s, slots, n);
    if (C > 0) hipLaunchKernelGGL(k_hash_insert, dim3((C + 255) / 256), dim3(256), 0, s, C, rows, slots, hbits);
    return hipGetLastError();
}

hipError_t launch_risk_measures(const float* y, int64_t n, const uint32_t* k_host, int32_t n_rp, const SelectWs& ws,
                                hipStream_t s)
{
    KList ks{};
    for (int r = 0; r < n_rp; ++r) ks.k[r] = k_host[r];
    const int nblk = (int)std::min<int64_t>(kSelectBlocks, std::max<int64_t>(1, (n + 255) / 256));
    hipLaunchKernelGGL(k_rm_init, dim3(1), dim3(256), 0, s, ws.state, ws.hist, ks, n_rp);
    for (int shift = 24; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_rm_hist, dim3(nblk), dim3(256), 0, s, y, n, n_rp, shift, (const uint32_t*)ws.state, ws.hist);
        hipLaunchKernelGGL(k_rm_pick, dim3(1), dim3(256), 0, s, ws.state, ws.hist, n_rp, shift);
    }
    hipLaunchKernelGGL(k_rm_tail, dim3(nblk), dim3(256), 0, s, y, n, n_rp, (const uint32_t*)ws.state, ws.partial);
    hipLaunchKernelGGL(k_rm_final, dim3(1), dim3(64), 0, s, (const uint32_t*)ws.state, (const double*)ws.partial, nblk,
                       ks, n_rp, ws.out);
    return hipGetLastError();
}

}  // namespace ara
