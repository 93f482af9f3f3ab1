// ara_internal.hpp -- device-side descriptors shared by the HIP kernels and
// the host half of libara (not part of the public ABI).
#pragma once

#include "ara_math.hpp"

namespace ara {

constexpr int kMaxEltsPerLayer = 64;
constexpr int kModeTable = 3;              // ARA_MODE_TABLE: the layer kernel's tabulated-inverse variant
constexpr int kMaxRp = 16;
constexpr double kSigmaClamp = 0.999;      // sigma_beta <= 0.999 * sigma_beta_max (applied in FP64)

struct SurEntry;
struct MlpFrag;

// A loaded XELT as the kernels see it.
struct EltDev {
    const int32_t* idx;     // [C] entry of each event, -1 if absent (direct-access table)
    const EntryRec* ent;    // [n] Beta parameters per entry
    const float2* cw;       // [n] (c_I, c_C) weights of section 3.2, or null if sigma_C == 0
    const double* mean;     // [n] mean loss mu_l
    const SolveRec* solve;  // [n] FP32 solve records with their start tables
    const TabRec* tab;      // [n] tabulated-inverse records (built on the first table-mode run), or null
    double ded, lim, share; // financial terms I of the XELT
    int32_t n;
    int32_t pad;
};

// The fourth word of an event's row: the event's entry count in the layer
// (bits 0-6) and, for its first kRowPolBits entries in rank order, whether the
// entry is a small shape whose draws are deferred (bit 7 + rank), so the solve
// can be chosen without reading the entry.
constexpr int kRowPolBits = 25;
__host__ __device__ inline int row_count(uint32_t w) { return (int)(w & 127u); }

// The device compile marks the layer tables' pointers as global memory, so
// the kernels gather through global (not flat) loads, which leave the LDS
// counter alone; host code stores them through gptr().
#ifdef __HIP_DEVICE_COMPILE__
#define ARA_GLOBAL __attribute__((address_space(1)))
#else
#define ARA_GLOBAL
#endif
template <typename T>
inline const ARA_GLOBAL T* gptr(const T* p) { return (const ARA_GLOBAL T*)p; }

// One layer of a run: its tables (built per run on the device) and terms.
struct LayerDev {
    const ARA_GLOBAL uint4* rows;   // [C] {mask bits 0-31, mask bits 32-63, first packed entry, count | flags},
                            // or, when hbits > 0, 2^hbits hash slots of two uint4 each:
                            // {event id (-1 empty), mask bits 0-31, mask bits 32-63, first entry}, {count | flags}
    uint32_t hbits;         // log2 of the hashed table's slot count; 0 = direct access
    const ARA_GLOBAL EntryRec* pent;   // [sum n_j] entries packed by event, in the layer's XELT order
    const ARA_GLOBAL float2* pcw;      // [sum n_j] combine weights, or null
    const ARA_GLOBAL SolveRec* psol;   // [sum n_j] solve records, packed like pent (plain mode), or null
    const ARA_GLOBAL TermThr* pthr;    // [sum n_j] sampling modes: term_thresholds for the entry's XELT
    const ARA_GLOBAL TabRec* ptab;     // [sum n_j] tabulated-inverse records, packed like pent (table mode), or null
    const float* occ_tab;   // [C] mean mode: per-event loss net of I and occurrence terms
    const SurEntry* psur;   // [sum n_j] surrogate mode: per-entry features and base
    float* ylt;             // [trial_end - trial_begin]
    float* omax;            // [trial_end - trial_begin] or null
    float* yelt;            // per occurrence, in the YET's layout from row(trial_begin), or null
    int64_t yelt_base;      // row(trial_begin)
    float occR, occL, aggR, aggL;
    uint32_t prog;
    uint32_t seed;          // key word of this layer's random numbers
    int32_t J;
    float4 jt[kMaxEltsPerLayer];   // per-XELT (deductible, limit, share, 0)
};

// A YET as the kernels see it.
struct YetDev {
    const int32_t* ev;      // event ids
    const int64_t* offs;    // [N+1] or null for a fixed K
    int64_t N;
    int32_t K;
    int32_t C;
};

// ---- launchers (ara_kernels.hip) ----
hipError_t launch_elt_index(const int32_t* event_id, int32_t n, int32_t* idx, hipStream_t s);
hipError_t launch_elt_prepare(int32_t n, const double* mean, const double* sig_i, const double* sig_c,
                              const double* maxl, EntryRec* ent, float2* cw, hipStream_t s);
hipError_t launch_elt_solve(int32_t n, const EntryRec* ent, SolveRec* sol, hipStream_t s);
hipError_t launch_validate_ids(const int32_t* ev, int64_t n, int32_t C, unsigned int* bad, hipStream_t s);
hipError_t launch_layer_count(int32_t C, int32_t J, const EltDev* elts, uint4* rows, uint32_t* cnt, hipStream_t s);
size_t scan_scratch_words(int64_t n);
hipError_t launch_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* scratch, hipStream_t s);
hipError_t launch_layer_fill(int32_t C, int32_t J, const EltDev* elts, const uint32_t* off, uint4* rows,
                             EntryRec* pent, float2* pcw, SolveRec* psol, TermThr* pthr, TabRec* ptab,
                             hipStream_t s);
hipError_t launch_elt_tab(int32_t n, const EntryRec* ent, TabRec* tab, hipStream_t s);
hipError_t launch_layer_hash(int32_t C, const uint4* rows, uint4* slots, uint32_t hbits, hipStream_t s);
hipError_t launch_beta_quantile_table(const double* a, const double* b, const double* u, int64_t n, double* x,
                                      hipStream_t s);
hipError_t launch_mean_table(int32_t C, int32_t J, const EltDev* elts, double occR, double occL,
                             float* occ_tab, hipStream_t s);
// wpb: wavefronts (= trials) per workgroup, 1, 2, 4 or 8 -- the trial tile
// Mean mode: catalog slices of the per-event table in LDS over a slice-major
// copy of the YET (mean_slices() == 0: too many slices, the table is read
// through L2 instead).  Group (slice s, trial t) of the copy starts at
// off[s * N + t] and holds cnt[s * N + t] ids (a multiple of 4, -1 padded);
// the copy holds at most T + 3 * ns * N ids for T ids in the YET.  The
// workspace holds each slice's per-trial partial sums and maxima.
int32_t mean_slices(int32_t C);
size_t mean_workspace_bytes(int32_t C, int64_t n_trials);
hipError_t launch_yet_slice_count(const YetDev& y, uint32_t* cnt, hipStream_t s);
hipError_t launch_yet_slice_scatter(const YetDev& y, const uint32_t* off, const uint32_t* cnt, uint16_t* ev2,
                                    hipStream_t s);
hipError_t launch_mean(const YetDev& y, int64_t t0, int64_t t1, const LayerDev* layers, int32_t n_layers,
                       const uint16_t* ev2, const uint32_t* goff, const uint32_t* gcnt, void* ws, bool yelt,
                       hipStream_t s);
// Per-occurrence aggregate increments of trials [t0, t1): occ and inc hold
// the trials' occurrences from row `base` of the YET on.
hipError_t launch_yelt_increments(const YetDev& y, int64_t t0, int64_t t1, int64_t base, double aggR, double aggL,
                                  const float* occ, float* inc, hipStream_t s);
hipError_t launch_layers(int mode, bool has_corr, const YetDev& y, int64_t t0, int64_t t1,
                         const LayerDev* layers, int32_t n_layers, int32_t wpb, hipStream_t s);

// ---- surrogate (ara_surrogate.hip) ----
hipError_t launch_sur_entries(const EntryRec* pent, int64_t n, SurEntry* psur, hipStream_t s);
hipError_t launch_layers_surrogate(bool has_corr, const YetDev& y, int64_t t0, int64_t t1, const LayerDev* layers,
                                   int32_t n_layers, const MlpFrag* frag, const uint32_t* cellmask,
                                   const float* bias, int32_t wpb,
                                   hipStream_t s);

hipError_t launch_philox_uniforms(const uint32_t* ctr, int64_t n, uint32_t k0, uint32_t k1, float* out, hipStream_t s);
hipError_t launch_beta_quantile_layer(const double* a, const double* b, const double* u, int64_t n, double* x,
                                      hipStream_t s);
hipError_t launch_beta_quantile(const double* a, const double* b, const double* u, int64_t n, double* x, hipStream_t s);

struct SelectWs {
    uint32_t* hist;         // [kMaxRp][256]
    uint32_t* state;        // [2*kMaxRp]: prefix key, remaining rank
    double* partial;        // [kSelectBlocks][kMaxRp]
    double* out;            // [2*kMaxRp]: pml, tvar
};
constexpr int kSelectBlocks = 256;
hipError_t launch_normal_quantile(const double* p, int64_t n, double* x, hipStream_t s);
hipError_t launch_sum_ylts(const float* const* ylts_dev, int32_t n, int64_t nt, float* out, hipStream_t s);
hipError_t launch_risk_measures(const float* y, int64_t n, const uint32_t* k_host, int32_t n_rp,
                                const SelectWs& ws, hipStream_t s);

}  // namespace ara
