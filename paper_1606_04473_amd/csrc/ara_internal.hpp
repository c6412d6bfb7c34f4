// Internal declarations shared by the HIP translation units of libara.
// Device code is written for gfx950 (CDNA4): 64-lane wavefronts, 160 KB LDS
// per CU, 256 CUs in 8 XCDs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "ara.h"

namespace ara {

constexpr int kWave = 64;

// The library's device memory (ara_api.hip): dev_alloc takes a block for work
// on stream s; dev_free gives it back after the work enqueued on s so far.  A
// block freed on s serves later work on s at once and work on other streams
// once s has reached the free.  Blocks are kept, not returned to the runtime.
hipError_t dev_alloc(void** p, size_t bytes, hipStream_t s);
void dev_free(void* p, hipStream_t s);
// bytes the cache of `device` holds, and of those not in use
void cache_stats(int device, int64_t* held, int64_t* idle);
// hipFree of the idle blocks of `device` whose last use has completed
int64_t cache_release(int device);
constexpr int kMaxJ = ARA_MAX_LAYER_ELTS;
constexpr int kStride = ARA_CHECKPOINT_EVERY;
// The event-ID array is padded with zero IDs so that aligned 16-byte loads
// covering a trial's last events never leave the allocation.
constexpr int64_t kIdPad = 1024;

// Layer description passed by value: it lands in the kernel-argument
// segment and is read with scalar loads (the paper kept financial terms in
// constant memory for the same reason: every lane reads the same value).
struct LayerArgs {
    int32_t J;
    int32_t pad_;
    double occR, occL, aggR, aggL;
    int64_t trial_begin, trial_count;
    int64_t out_offset;
    int32_t idx[kMaxJ];
    double R[kMaxJ];
    double Lim[kMaxJ];
};

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

// clamp(v; r, lim) = min(max(v - r, 0), lim): retention r, then limit lim.
__device__ __forceinline__ double apply_terms(double v, double r, double lim) {
    double t = v - r;
    t = (t > 0.0) ? t : 0.0;
    t = (t > lim) ? lim : t;
    return t;
}

// Error-free sum (Knuth): s + e == a + b exactly.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Double-double accumulate: (hi, lo) += x.
__device__ __forceinline__ void dd_add(double& hi, double& lo, double x) {
    double s, e;
    two_sum(hi, x, s, e);
    hi = s;
    lo += e;
}

// (hi, lo) += (hi2, lo2).  Symmetric in its operands, so butterfly partners
// end with identical values.
__device__ __forceinline__ void dd_merge(double& hi, double& lo, double hi2, double lo2) {
    double s, e;
    two_sum(hi, hi2, s, e);
    hi = s;
    lo = (lo + lo2) + e;
}

__device__ __forceinline__ double shfl_xor_f64(double v, int mask) {
    return __shfl_xor(v, mask, kWave);
}

__device__ __forceinline__ double shfl_f64(double v, int src) {
    return __shfl(v, src, kWave);
}

// Butterfly reduction over `width` lanes (power of two <= 64); every lane of
// each group of `width` lanes ends with the group's total.
__device__ __forceinline__ void group_reduce_dd(double& hi, double& lo, int width) {
    for (int off = width >> 1; off >= 1; off >>= 1) {
        double h2 = shfl_xor_f64(hi, off);
        double l2 = shfl_xor_f64(lo, off);
        dd_merge(hi, lo, h2, l2);
    }
}

__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
    uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
    uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(static_cast<uint64_t>(v) >> 32));
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// host-side state
// ---------------------------------------------------------------------------

struct CheckpointState {
    bool valid = false;
    LayerArgs key{};
    double* S = nullptr;        // [trial_count]
    double* ylt = nullptr;      // [trial_count]
    double* stride = nullptr;   // [n_events / 64 + 1]
    bool has_stride = false;
    int64_t count = 0;
};

// Part-major copy of the YET (see kernels_parts.hip): tiles of T trials,
// inside a tile part by part, inside a part trial by trial.
constexpr int kMaxParts = 64;

// The nonzero entries of the ELT pool, row by row in 4096-event chunks (one
// superblock of the part images each): entries of chunk c of row r are
// [chunk_off[r * n_chunks + c], chunk_off[r * n_chunks + c + 1]), in event
// order, with the event's index inside the chunk and its loss.
struct SparsePool {
    uint16_t* ev = nullptr;         // event index within its chunk
    double* val = nullptr;          // loss (> 0)
    int64_t* chunk_off = nullptr;   // [n_rows * n_chunks + 1]
    int64_t n_chunks = 0;
    int64_t nnz = 0;
    int64_t bytes = 0;
};
hipError_t build_sparse_pool(const double* elts, int32_t n_rows, int64_t C, hipStream_t s, SparsePool* out);
void free_sparse_pool(SparsePool* sp);
struct PartLayout {
    int P = 0;                      // catalogue parts; 0 = layout absent
    int T = 0;                      // trials per tile
    int64_t n_tiles = 0;
    int64_t length = 0;             // IDs in pids (with padding)
    int64_t bytes = 0;
    uint32_t* pids = nullptr;       // [length + kIdPad]
    uint32_t* seg_rel = nullptr;    // [n_tiles][T*P + 1] segment starts relative to the tile
    int64_t* tile_start = nullptr;  // [n_tiles + 1]
};

// Per-request part images, one per 2^18-event part of the catalogue, written
// by launch_fold_parts at the start of the part scratch: u64 bitmap words of
// o(E) != 0, a u16 rank per 128 events relative to its 4096-event
// superblock, and the u32 global rank of each superblock.  The nonzero o(E)
// themselves follow, in rank order (part_compact_values).
constexpr int kImgShift = 18;
constexpr int kImgWords = (1 << kImgShift) / 64;
constexpr int kImgRank16 = (1 << kImgShift) / 128;
constexpr int kImgBase32 = (1 << kImgShift) / 4096;
constexpr int64_t kImgPartBytes = int64_t(kImgWords) * 8 + int64_t(kImgRank16) * 2 + int64_t(kImgBase32) * 4;
double* part_compact_values(void* part_scratch, int P);
// nonzero o(E) per 4096-event superblock, P * 64 of them, after launch_fold_parts
uint32_t* part_superblock_counts(void* part_scratch, int P);

// Second copy of the YET for the streaming pass (kernels_stream.hip): the
// catalogue cut into parts of 2^16 events; per part, one contiguous stream of
// 16-bit part-relative IDs holding, group of G consecutive trials after
// group, each trial's events of that part in time order.  Groups start on
// 16-byte boundaries (the gap holds 0xFFFF).
constexpr int kStreamShift = 16;
constexpr int kMaxStreamParts = 64;
constexpr int kStreamGroupMax = 63;       // trials per group at most (one lane each, plus the group's end)
constexpr int kStreamGroupSlots = 64;     // trial ends kept per group (slots past the group's trials repeat its end)
struct StreamLayout {
    int P = 0;                      // stream parts; 0 = layout absent
    int G = 0;                      // trials per group (<= kStreamGroupMax)
    int64_t NG = 0;                 // groups: ceil(N / G)
    int64_t length = 0;             // IDs, padding included
    int64_t bytes = 0;
    uint16_t* ids = nullptr;        // [length + 8 * 64]
    int64_t* part_base = nullptr;   // [P + 1] first ID of each part's stream
    uint32_t* gstart = nullptr;     // [P][NG + 1] group starts relative to the part's stream
    uint16_t* gend = nullptr;       // [P][NG][64] end of trial i of the group, relative to the group start
};
hipError_t build_stream_layout(const int64_t* offsets, const uint32_t* ids, int64_t N, int64_t n_events, int64_t C,
                               int n_cu, hipStream_t s, StreamLayout* out);
// frees in stream order on s (the layout's memory comes from dev_alloc)
void free_stream_layout(StreamLayout* L, hipStream_t s);
// bytes of the per-(part, trial) partial sums of the streaming pass
int64_t stream_partials_bytes(const StreamLayout& lay, int64_t trials);
// the streaming pass: reads the part images and compact values that
// launch_fold_parts wrote to part_scratch (n_img_parts 2^18-event parts), writes
// per-(stream part, trial) partial sums; the combine merges them in part order
hipError_t launch_stream_pass(const StreamLayout& lay, int64_t C, const LayerArgs& L, void* part_scratch,
                              int n_img_parts, void* partials, int n_cu, hipStream_t s);
hipError_t launch_stream_combine(const StreamLayout& lay, const LayerArgs& L, const LayerArgs* L_dev,
                                 const void* partials, double* ylt, double* S, hipStream_t s);
struct TailStats;
// the backward histogram over the same stream: for the trials inside the
// aggregate band, occurrences of each nonzero-o(E) event added to w_mean and
// TVaR weights to w_tvar (both [C], zeroed by the caller); S and ylt are the
// checkpointed forward's, tail its order statistics on the device.  scratch
// holds stream_adjoint_scratch_bytes(L.trial_count) bytes.
int64_t stream_adjoint_scratch_bytes(int64_t trials);
hipError_t launch_stream_adjoint(const StreamLayout& lay, int64_t C, const LayerArgs& L, void* part_scratch,
                                 int n_img_parts, const double* S, const double* ylt, const TailStats* tail,
                                 void* scratch, int64_t scratch_bytes, uint64_t* w_mean, uint64_t* w_tvar, int n_cu,
                                 hipStream_t s);

constexpr int kXcds = 8;           // gfx950 (MI355X): 8 XCDs, workgroups dispatched round-robin

struct XcdPassArgs {
    const uint32_t* pids;
    const uint32_t* seg_rel;
    const int64_t* tile_start;
    const uint8_t* img;             // part images: bitmap, 128-event ranks, superblock bases
    const double* compact;          // nonzero occurrence losses in rank order
    int64_t C;                      // catalogue size (bounds compact)
    int64_t N;
    int P;
    int T;
    int64_t t_lo, t_hi;
    int64_t first_tile, last_tile;
    double* part_hi;                // [P][count]
    double* part_lo;
    const uint32_t* pad;            // 16 readable bytes of sentinels (the padding after the IDs)
    int n_xcd;
};

struct PartPassArgs {
    const uint32_t* pids;
    const uint32_t* seg_rel;
    const int64_t* tile_start;
    const uint8_t* img;
    const double* compact;
    int64_t N;
    int P;
    int T;
    int64_t t_lo, t_hi;
    int64_t first_tile, last_tile;
    double aggR, aggL;
    double* ylt;
    double* S;
    uint32_t* tile_counter;
};

// batched multi-layer pass
struct BatchLayerDesc {
    int64_t t_lo, t_hi;
    double aggR, aggL;
    int64_t out_off;
};
struct BatchFoldDesc {
    int32_t J, off;
    double occR, occL;
};
struct BatchedPassArgs {
    const uint32_t* pids;
    const uint32_t* seg_rel;
    const int64_t* tile_start;
    const uint8_t* img;
    int64_t img_stride;
    const double* compact;
    int64_t C;
    int64_t N;
    int P;
    int T;
    const int2* items;             // (layer, tile), decreasing cost
    int32_t n_items;
    const BatchLayerDesc* layers;
    double* ylt;
    uint32_t* item_counter;
};
struct BatchedScratch {
    double* o;
    double* compact;
    uint8_t* img;
    uint32_t* sb_count;
    uint32_t* counter;
    int2* items;
    BatchLayerDesc* layers;
    BatchFoldDesc* fold;
    double* R;
    double* Lim;
    int32_t* idx;
};

struct TailStats;
struct PartAdjArgs {
    const uint32_t* pids;
    const uint32_t* seg_rel;
    const int64_t* tile_start;
    const uint8_t* img;
    int64_t N;
    int P;
    int T;
    int64_t t_lo, t_hi;
    int64_t first_tile, last_tile;
    double aggR, aggL;
    const double* S;
    const double* ylt;
    const TailStats* tail;
    uint64_t* w_mean;
    uint64_t* w_tvar;
    uint32_t* tile_counter;
    const uint32_t* sb_count;       // nonzero count of each superblock (for part-relative ranks)
};

struct ProfileState {
    struct Pending {
        hipEvent_t start, stop;
        int kind;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> free_events;
    int64_t launches[5] = {0, 0, 0, 0, 0};
    double total_ms[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
};

// Pinned host staging for small per-call uploads; the event marks when the
// last copy out of it has completed.
struct HostStage {
    void* p = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
};

// Device scratch kept between calls.  Stream-ordered allocation makes the
// host wait for the previous call's work before it hands the memory out
// again; a kept buffer is handed to the next call on the same stream at once
// (stream order protects it), or to a call on another stream once the event
// recorded after its last use has completed.  Calls that find no free buffer
// get a new one, so concurrent callers never share.
struct ScratchBuffer {
    void* p = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;      // recorded on `stream` after the last use
    hipStream_t stream = nullptr;
    bool busy = false;
    bool primed = false;            // metrics: left ready by a whole launch sequence (cleared on growth)
};

// A captured batched run: persistent scratch, a graph, and the shape it was
// captured for.
struct GraphEntry {
    std::vector<int64_t> key;
    void* scratch = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    HostStage stage;
    std::vector<uint8_t> last;          // the layer arguments last copied to `scratch`,
    hipStream_t last_stream = nullptr;  // on this stream (stage.done marks the copy)
};

}  // namespace ara

struct ara_tables {
    int device = 0;
    int n_cu = 256;
    int64_t n_trials = 0;
    int64_t n_events = 0;
    int64_t C = 0;
    int32_t n_pool = 0;
    int64_t* offsets = nullptr;   // [n_trials + 1]
    uint32_t* ids = nullptr;      // [n_events + kIdPad]
    double* elts = nullptr;       // [n_pool][C]
    bool owns_elts = true;        // false: the pool belongs to another tables object
    ara::SparsePool sparse;       // the pool's nonzero entries (shared with the pool's owner)
    int64_t bytes = 0;
    ara_tuning tuning{};
    std::mutex mu;                // guards ck and tuning
    ara::CheckpointState ck;
    ara::PartLayout parts;
    ara::StreamLayout stream;     // 16-bit part-major copy for the streaming pass
    std::mutex stage_mu;          // guards stage and graphs
    ara::HostStage stage;
    std::vector<ara::GraphEntry*> graphs;
    std::mutex prof_mu;           // guards prof
    ara::ProfileState prof;
    std::mutex scratch_mu;        // guards scratch
    std::vector<ara::ScratchBuffer*> scratch;
    // one event per stream the tables were used on, recorded after each call's
    // work: destroying the tables returns their memory to the cache after all
    // of them, without waiting on the host
    std::mutex fence_mu;
    std::vector<std::pair<hipStream_t, hipEvent_t>> fences;
};

namespace ara {

// ---------------------------------------------------------------------------
// launchers (each defined in the translation unit holding its kernels)
// ---------------------------------------------------------------------------

struct TrialPassArgs {
    const int64_t* offsets;
    const uint32_t* ids;
    const double* elts;   // literal mode
    int64_t C;
    const double* o;      // folded mode: occurrence-net loss per catalogue event
    double* ylt;          // [trial_count]
    double* S;            // [trial_count] or null
    double* stride;       // checkpoints or null
};

hipError_t launch_validate(const int64_t* offsets, int64_t n_trials, const uint32_t* ids,
                           int64_t n_events, const double* elts, int64_t n_elt_values,
                           int64_t C, uint32_t* d_flags, int n_cu, hipStream_t s);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s);

hipError_t launch_fold(const double* elts, int64_t C, const LayerArgs& L, double* o,
                       const ara_tuning& tu, hipStream_t s);
hipError_t launch_trial_pass(const TrialPassArgs& a, const LayerArgs& L, bool literal,
                             const ara_tuning& tu, int n_cu, hipStream_t s);
// per-trial sums of layer year losses into program and portfolio year losses
struct PortfolioSumArgs {
    const double* layer_ylt;              // [n_layers][count]
    int64_t count;
    int32_t n_programs;
    int32_t first[ARA_MAX_PROGRAMS + 1];  // program p sums layers [first[p], first[p + 1])
    double* program_ylt;                  // [n_programs][count] or null
    double* portfolio_ylt;                // [count] or null
};
hipError_t launch_portfolio_sum(const PortfolioSumArgs& a, int n_cu, hipStream_t s);
// per-event net losses of a layer's trials, in time order, reading o(E)
// through the part images and compact values that launch_fold_parts wrote to
// part_scratch (P = catalogue parts)
hipError_t launch_event_nets(const int64_t* offsets, const uint32_t* ids, const void* part_scratch, int P,
                             int64_t C, uint64_t* probe, const LayerArgs& L, double* nets, int n_cu, hipStream_t s);
// the forward's stride checkpoints in the same time-ordered pass: slot b of
// `stride` receives the running total S of the trial that owns global event
// 64b + 63, after that event (slots outside the layer's trials untouched)
hipError_t launch_stride_checkpoints(const int64_t* offsets, const uint32_t* ids, const void* part_scratch, int P,
                                     int64_t C, uint64_t* probe, const LayerArgs& L, double* stride, int n_cu,
                                     hipStream_t s);
int64_t probe_table_bytes(int64_t C);   // scratch for launch_event_nets' probe words
hipError_t launch_debug_lookups(const int64_t* offsets, const uint32_t* ids, const double* elts,
                                int64_t C, const LayerArgs& L, int64_t trial, uint32_t* ids_out,
                                double* losses_out, hipStream_t s);

// catalogue-partitioned path
hipError_t build_part_layout(const int64_t* offsets, const uint32_t* ids, int64_t N, int64_t n_events, int64_t C,
                             int n_cu, hipStream_t s, PartLayout* out);
// frees in stream order on s (the layout's memory comes from dev_alloc)
void free_part_layout(PartLayout* L, hipStream_t s);
int64_t part_scratch_bytes(int64_t C, int P);
int part_count(int64_t C);   // catalogue parts of the part images
hipError_t launch_part_fold(const double* o, int64_t C, int P, void* scratch, hipStream_t s, bool with_ranks);
// the fold fused with the part images, then ranks and the compact array; with
// L_dev the terms are read from device memory (for graph replays), else from L
hipError_t launch_fold_parts(const SparsePool& sp, int64_t C, const LayerArgs& L, const LayerArgs* L_dev, double* o,
                             int P, void* scratch, hipStream_t s);
// the XCD-affine pass writes per-part partial sums; the combine merges them
hipError_t launch_xcd_pass(const PartLayout& lay, int64_t N, int64_t C, const LayerArgs& L, void* part_scratch,
                           double* partials, int n_cu, hipStream_t s);
hipError_t launch_xcd_combine(const PartLayout& lay, const LayerArgs& L, const LayerArgs* L_dev,
                              const double* partials, double* ylt, double* S, hipStream_t s);
hipError_t launch_part_pass(const PartLayout& lay, int64_t N, const LayerArgs& L, void* scratch, double* ylt,
                            double* S, int n_cu, hipStream_t s, int lpt);

int64_t batched_scratch_bytes(int64_t C, int P, int n_layers, int64_t n_items, int64_t n_elts_total);
BatchedScratch carve_batched(void* scratch, int64_t C, int P, int n_layers, int64_t n_items, int64_t n_elts_total);
hipError_t launch_batched(const PartLayout& lay, int64_t N, int64_t C, const double* elts, int n_layers,
                          const BatchedScratch& b, int64_t n_items, double* ylt, int n_cu, hipStream_t s,
                          hipEvent_t pass_start, hipEvent_t pass_stop, int lpt);

// metrics: *mean, pml[q * stride] = PML_q, tvar[q * stride] = TVaR_q (device pointers)
struct MetricsOut {
    double* mean;
    double* pml;
    double* tvar;
    int stride;
};
// scratch of launch_metrics for n_probs probabilities over n year losses
int64_t metrics_scratch_bytes(int n_probs, int64_t n);
// `primed`: the scratch was last used by a launch_metrics sequence that was
// enqueued whole, which leaves it ready for the next one (no init kernel)
// readies a new scratch for launch_metrics(..., primed = true): the state the
// previous sequence of a reused scratch leaves behind
hipError_t launch_metrics_prime(void* scratch, const int64_t* m_host, int n_probs, hipStream_t s);
hipError_t launch_metrics(const double* ylt, int64_t n, const int64_t* m_host, int n_probs,
                          void* scratch, bool primed, MetricsOut out, int n_cu, hipStream_t s);

// the static scratch of ara_risk_metrics_noalloc on the current device and
// its size in bytes (launch_metrics needs metrics_scratch_bytes of it)
hipError_t metrics_noalloc_scratch(void** ptr, int64_t* capacity);

// order statistics of a YLT for one tail count m
struct TailStats {
    uint64_t v_bits;   // bit pattern of the m-th largest year loss
    int64_t c_gt;      // year losses strictly above it
    int64_t c_eq;      // year losses equal to it
    int64_t m;
};
int64_t tail_stats_scratch_bytes(int64_t n);
hipError_t launch_tail_stats(const double* ylt, int64_t n, int64_t m, void* scratch, TailStats* out,
                             int n_cu, hipStream_t s);

hipError_t launch_part_adjoint(const PartLayout& lay, int64_t N, const LayerArgs& L, void* part_scratch,
                               const double* S, const double* ylt, const TailStats* tail, uint64_t* w_mean,
                               uint64_t* w_tvar, int n_cu, hipStream_t s);

// adjoint; with `parts` (and `part_scratch` holding the forward's part images)
// the histogram pass runs over the partitioned layout, or over the 16-bit
// stream when `stream` is given and holds one
int64_t adjoint_scratch_bytes(int64_t C, int J, int64_t n);
hipError_t launch_adjoint(const int64_t* offsets, const uint32_t* ids, const double* elts,
                          int64_t C, const LayerArgs& L, const double* S, const double* ylt,
                          int64_t m, void* scratch, double* d_grad_mean, double* d_grad_tvar,
                          int n_cu, hipStream_t s, const PartLayout* parts, void* part_scratch,
                          int64_t n_trials_total, const SparsePool* sp, const StreamLayout* stream);

}  // namespace ara
