// Streaming trial pass over a 16-bit, part-major copy of the YET.
//
// Algorithm 3 reduces, after the per-request fold (o(E) for every catalogue
// event: the per-ELT terms, the combination over ELTs and the occurrence
// terms, which depend on the event alone), to S_t = sum of o(E) over the
// events of trial t, then the aggregate terms.  Most o(E) are zero, so the
// work per streamed event is one question -- is o(E) nonzero, and what is it
// -- answered here entirely from LDS:
//
//  * the catalogue is cut into parts of 2^16 events.  At table creation the
//    YET is copied part-major: for each part one contiguous stream holding,
//    group of G consecutive trials after group, each trial's events of that
//    part in time order, as 16-bit part-relative IDs.  Each group starts on
//    a 16-byte boundary (the gap holds 0xFFFF), and the end of every trial
//    inside its group is kept as a 16-bit offset.  The stream is half the
//    bytes of the 32-bit IDs.
//  * a workgroup (16 waves, one per CU) takes a contiguous run of (part,
//    group) work items.  For its part it builds in LDS a byte per catalogue
//    event -- 0 for o(E) = 0, else 1 + the event's rank among the nonzero
//    events of its 128-event block -- plus the rank of each block's first
//    nonzero event, and copies the part's first nonzero o(E) (in rank order)
//    into the rest of its LDS.  One ID costs one address operation and one
//    LDS byte read.
//  * each wave streams one group (up to 63 trials) in batches of two 16-byte
//    loads per lane, the next batch in flight while this one is tested, and
//    appends the hits in stream order to its LDS queue.  Lane i holds where
//    trial i starts; the queue index of its first hit comes from the
//    per-chunk hit masks.  At the end of the group lane t sums trial t's
//    queued losses in double-double, in queue order, so the result does not
//    depend on timing.
//  * each (part, trial) partial sum is written once (high part FP64, low part
//    FP32); the combine adds a trial's partials in part order, rounds once and
//    applies the aggregate terms.
//  * the backward's histogram (how often each event with o(E) != 0 occurs in
//    the trials inside the aggregate band, and the TVaR weights of the tail
//    trials) is the same kernel instantiated with kAdj: the same test and
//    queue, a drain that counts occurrences in LDS instead of summing losses.
#include <cmath>
#include <vector>

#include "ara_internal.hpp"

namespace ara {

namespace {

constexpr int kQSize = 1 << kStreamShift;       // catalogue events per stream part
constexpr int kChunkIds = 8;                    // 16-bit IDs per 16-byte load
constexpr int64_t kStreamPad = 512;             // readable 0xFFFF IDs after the stream

__device__ __forceinline__ uint64_t stream_lanemask_lt() {
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// ---------------------------------------------------------------------------
// create-time layout
// ---------------------------------------------------------------------------

// cnt[t * P + q] = events of trial t in stream part q; one wave per trial
__global__ __launch_bounds__(256) void stream_count_kernel(const int64_t* __restrict__ offsets,
                                                           const uint32_t* __restrict__ ids, int64_t N, int P,
                                                           int32_t* __restrict__ cnt) {
    __shared__ int32_t c[4][kMaxStreamParts];
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t n_waves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
    for (int64_t t = uniform_i64((static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6); t < N;
         t += n_waves) {
        for (int p = lane; p < P; p += 64) c[w][p] = 0;
        __builtin_amdgcn_wave_barrier();
        {
            // four 64-ID chunks loaded together
            const int64_t b = offsets[t], e = offsets[t + 1];
            for (int64_t c0 = b; c0 < e; c0 += 256) {
                uint32_t idk[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int64_t at = c0 + k * 64 + lane;
                    idk[k] = at < e ? ids[at] : 0u;
                }
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (c0 + k * 64 + lane < e) atomicAdd(&c[w][idk[k] >> kStreamShift], 1);
            }
        }
        __builtin_amdgcn_wave_barrier();
        for (int p = lane; p < P; p += 64) cnt[t * P + p] = c[w][p];
        __builtin_amdgcn_wave_barrier();
    }
}

// per (part, group) k = q * NG + g: the end of each of the group's trials
// relative to the group start (slots past the group's trials repeat the
// group's end), and the group's size padded to whole 16-byte chunks.  Flags
// bit 0 when a group holds more than 65535 IDs of one part.
__global__ __launch_bounds__(256) void stream_group_kernel(const int32_t* __restrict__ cnt, int64_t N, int P, int G,
                                                           int64_t NG, uint16_t* __restrict__ gend,
                                                           uint32_t* __restrict__ gsize, uint32_t* __restrict__ flag) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= static_cast<int64_t>(P) * NG) return;
    const int q = static_cast<int>(k / NG);
    const int64_t g = k - static_cast<int64_t>(q) * NG;
    uint32_t run = 0;
    for (int i = 0; i < kStreamGroupSlots; ++i) {
        const int64_t t = g * G + i;
        if (i < G && t < N) run += static_cast<uint32_t>(cnt[t * P + q]);
        gend[k * kStreamGroupSlots + i] = static_cast<uint16_t>(run < 65535u ? run : 65535u);
    }
    if (run > 65535u) atomicOr(flag, 1u);
    gsize[k] = (run + kChunkIds - 1) & ~static_cast<uint32_t>(kChunkIds - 1);
}

// per part (one workgroup each): exclusive scan of the padded group sizes;
// flags bit 1 when a part's stream reaches 2^32 IDs
__global__ __launch_bounds__(1024) void stream_scan_kernel(const uint32_t* __restrict__ gsize, int64_t NG,
                                                           uint32_t* __restrict__ gstart,
                                                           uint64_t* __restrict__ part_len,
                                                           uint32_t* __restrict__ flag) {
    __shared__ uint64_t tsum[1024];
    const int q = blockIdx.x;
    const uint32_t* src = gsize + static_cast<int64_t>(q) * NG;
    uint32_t* dst = gstart + static_cast<int64_t>(q) * (NG + 1);
    const int64_t per = (NG + 1023) / 1024;
    const int64_t j0 = static_cast<int64_t>(threadIdx.x) * per;
    uint64_t local = 0;
    for (int64_t j = j0; j < j0 + per && j < NG; ++j) local += src[j];
    tsum[threadIdx.x] = local;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint64_t add = static_cast<int>(threadIdx.x) >= off ? tsum[threadIdx.x - off] : 0ull;
        __syncthreads();
        tsum[threadIdx.x] += add;
        __syncthreads();
    }
    uint64_t run = tsum[threadIdx.x] - local;
    for (int64_t j = j0; j < j0 + per && j < NG; ++j) {
        dst[j] = static_cast<uint32_t>(run);
        run += src[j];
    }
    if (threadIdx.x == 1023) {
        const uint64_t total = tsum[1023];
        dst[NG] = static_cast<uint32_t>(total);
        part_len[q] = total;
        if (total >= (uint64_t(1) << 32) - 4096) atomicOr(flag, 2u);
    }
}

__global__ void stream_fill_kernel(uint32_t* p, int64_t n, uint32_t v) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Stable scatter of each trial's events into its segments of the part
// streams, one workgroup per group of G trials.  The group's segments of
// every part are staged in LDS (each padded with 0xFFFF as in the stream) and
// its trials are scattered there, one wave per trial, sixteen at a time: for
// each 64 events every lane finds the lanes holding an event of its own part
// -- the AND over the part number's bits of that bit's ballot or its
// complement -- takes its rank among the earlier ones, and all 64 write in
// one store; the last lane of each part moves that part's cursor on.  Each
// part's segment then leaves in 16-byte stores to its place in the stream:
// whole lines instead of 2-byte writes spread over up to P lines per 64
// events.  A group whose padded segments exceed the stage is scattered
// straight to the stream.
constexpr int kGroupStageIds = 72 * 1024;     // 144 KB of LDS
__global__ __launch_bounds__(1024) void stream_group_scatter_kernel(
    const int64_t* __restrict__ offsets, const uint32_t* __restrict__ ids, int64_t N, int P, int G, int64_t NG,
    const int64_t* __restrict__ part_base, const uint32_t* __restrict__ gstart, const uint16_t* __restrict__ gend,
    uint16_t* __restrict__ out) {
    __shared__ __attribute__((aligned(16))) uint16_t stage[kGroupStageIds];
    __shared__ uint32_t seg[kMaxStreamParts + 1];     // staged start of each part's segment
    __shared__ int64_t cur[16][kMaxStreamParts];       // per wave: where each part's next event goes
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int n_bits = P > 1 ? 32 - __builtin_clz(static_cast<uint32_t>(P - 1)) : 0;
    const uint64_t below = stream_lanemask_lt();
    const uint64_t above = lane == 63 ? 0ull : (~0ull << (lane + 1));
    for (int64_t g = blockIdx.x; g < NG; g += gridDim.x) {
        if (w == 0) {                                  // each part's padded segment, scanned over the wave
            uint32_t n = 0;
            if (lane < P) {
                const int64_t k = static_cast<int64_t>(lane) * (NG + 1) + g;
                n = gstart[k + 1] - gstart[k];
            }
            uint32_t inc = n;
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t v = __shfl_up(inc, off, 64);
                if (lane >= off) inc += v;
            }
            if (lane < P) seg[lane] = inc - n;
            if (lane == P - 1) seg[P] = inc;
        }
        __syncthreads();
        const uint32_t total = seg[P];
        const bool staged = total <= static_cast<uint32_t>(kGroupStageIds);
        if (staged) {
            for (uint32_t u = threadIdx.x; u < total / 8; u += blockDim.x)
                reinterpret_cast<u32x4*>(stage)[u] = u32x4{0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
        }
        __syncthreads();
        const int64_t t0 = g * G;
        const int64_t t1 = t0 + G < N ? t0 + G : N;
        for (int64_t t = t0 + w; t < t1; t += 16) {
            const int i = static_cast<int>(t - t0);
            for (int q = lane; q < P; q += 64) {
                const int64_t k = static_cast<int64_t>(q) * NG + g;
                const int64_t rel = i ? gend[k * kStreamGroupSlots + i - 1] : 0;
                cur[w][q] = staged ? seg[q] + rel
                                   : part_base[q] + gstart[static_cast<int64_t>(q) * (NG + 1) + g] + rel;
            }
            __builtin_amdgcn_wave_barrier();
            const int64_t b = offsets[t], e = offsets[t + 1];
            constexpr int kAhead = 8;                   // chunks of 64 IDs loaded together
            for (int64_t c0 = b; c0 < e; c0 += 64 * kAhead) {
                uint32_t idk[kAhead];
#pragma unroll
                for (int k = 0; k < kAhead; ++k) {
                    const int64_t at = c0 + k * 64 + lane;
                    idk[k] = at < e ? ids[at] : 0u;
                }
#pragma unroll
                for (int k = 0; k < kAhead; ++k) {
                    const int64_t c = c0 + k * 64;
                    if (c >= e) break;
                    const bool valid = c + lane < e;
                    const uint32_t id = idk[k];
                    const int pid = static_cast<int>(id >> kStreamShift);
                    uint64_t same = __ballot(valid);
                    for (int bit = 0; bit < n_bits; ++bit) {
                        const bool set = ((pid >> bit) & 1) != 0;
                        const uint64_t lanes = __ballot(set);
                        same &= set ? lanes : ~lanes;
                    }
                    const int64_t at = cur[w][pid];
                    if (valid) {
                        const int64_t to = at + __popcll(same & below);
                        if (staged)
                            stage[to] = static_cast<uint16_t>(id);
                        else
                            out[to] = static_cast<uint16_t>(id);
                    }
                    __builtin_amdgcn_wave_barrier();
                    if (valid && (same & above) == 0) cur[w][pid] = at + __popcll(same);
                    __builtin_amdgcn_wave_barrier();
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        if (staged) {
            // segments are whole 8-ID chunks, here and in the stream
            for (int q = w; q < P; q += 16) {
                const uint32_t s0 = seg[q] / 8, s1 = seg[q + 1] / 8;
                u32x4* dst = reinterpret_cast<u32x4*>(out + part_base[q] +
                                                      gstart[static_cast<int64_t>(q) * (NG + 1) + g]);
                for (uint32_t u = s0 + lane; u < s1; u += 64) dst[u - s0] = reinterpret_cast<const u32x4*>(stage)[u];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// the pass
// ---------------------------------------------------------------------------

struct StreamPassArgs {
    const uint16_t* ids;
    const int64_t* part_base;
    const uint32_t* gstart;
    const uint16_t* gend;
    const uint8_t* img;             // part images of the 2^18-event parts
    const double* compact;          // nonzero o(E) in rank order
    int64_t C;
    int P;
    int G;
    int64_t NG;
    int64_t g_lo, g_hi;             // groups holding the layer's trials
    int64_t t_lo, t_hi;
    double* part_hi;                // [P][t_hi - t_lo]
    float* part_lo;
    const uint16_t* pad;            // 16 readable bytes of 0xFFFF
    int n_xcd;
};

// bit if the lane's condition holds, else 0: one select on the compare's lane
// mask, so the compare that also guards the lane's queue append is not redone
// in inverted form
template <uint32_t kBit>
__device__ __forceinline__ uint32_t lane_select(bool cond) {
    const uint64_t lanes = __builtin_amdgcn_ballot_w64(cond);
    uint32_t r;
    if constexpr (kBit <= 64)                   // an inline constant
        __asm__("v_cndmask_b32_e64 %0, 0, %1, %2" : "=v"(r) : "i"(kBit), "s"(lanes));
    else
        __asm__("v_cndmask_b32_e64 %0, 0, %1, %2" : "=v"(r) : "v"(kBit), "s"(lanes));
    return r;
}

// Inclusive prefix sum over the 64 lanes of a wave: four DPP row shifts, then
// two row broadcasts carry the row totals.
__device__ __forceinline__ uint32_t stream_wave_scan(uint32_t x) {
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x111, 0xF, 0xF, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x112, 0xF, 0xF, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x114, 0xF, 0xF, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x118, 0xF, 0xF, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x142, 0xA, 0xF, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x143, 0xC, 0xF, false));
    return x;
}

// Extra arguments of the backward histogram over the stream.  Lane i of group
// g holds trial g*G + i's class: 0 outside the layer's trials or outside the
// aggregate band, else bit 0, plus bit 1 when its year loss lies above the
// m-th largest (TVaR weight c_eq) or bit 2 when it equals it (weight m - c_gt)
struct StreamAdjArgs {
    const uint8_t* cls;             // [g_hi - g_lo][64]
    uint64_t* w_mean;               // [C] occurrences in trials inside the band
    uint64_t* w_tvar;               // [C] TVaR weights
    const TailStats* tail;
};

// The pass over the stream.  The forward (kAdj false) sums each trial's
// nonzero o(E), part by part.  The backward histogram (kAdj true) runs the
// same test and queue; its drain counts each queued occurrence of a trial
// inside the aggregate band per event, in 32-bit LDS counters indexed by rank
// that go to W_mean when the workgroup leaves the part (ranks past the
// counters, and the TVaR weights of the few tail trials, use global atomics).
// All weights are integers, so the order of the additions does not matter.
//
// gstart_all is a.gstart again, as a restrict-qualified parameter: its loads at
// wave-uniform addresses then go through the scalar unit, so a group's range
// never waits on the vector loads in flight
template <bool kAdj>
__global__ __launch_bounds__(1024) void stream_pass_kernel(StreamPassArgs a, StreamAdjArgs adj,
                                                           const uint32_t* __restrict__ gstart_all) {
    constexpr int kU = 2;                                     // 16-byte loads per lane per batch
    constexpr uint32_t kBatch = 64 * kChunkIds * kU;          // IDs per batch
    constexpr int kQ = 64 * kChunkIds;                        // 16-bit queue entries per wave: one load's IDs
    constexpr int kInf = 0x3FFFFFFF;
    constexpr int kHeld = 4;                                  // groups' sums held before a store
    // s_waitcnt operand: vector memory count 0, the other counters at their maximum
    constexpr int kWaitVm0 = (0xF << 8) | (0x7 << 4);
    static_assert(kU == 2, "a batch is two loads per lane, each fitting an empty queue");
    // LDS, one block: the rank of each 128-event block's first nonzero event
    // minus one, then the byte map (a byte's offset from the map's start is its
    // event's part-relative ID; that offset fits the LDS instructions' constant
    // field, so a lookup costs no address arithmetic), the 16 hit queues, and
    // then the forward's copy of as many of the part's nonzero o(E) as fit,
    // followed by one 0.0 that the drain's idle slots read, or the backward's
    // counters
    constexpr uint32_t kMapOff = (kQSize / 128) * 4;
    constexpr uint32_t kQueueOff = kMapOff + kQSize;
    constexpr uint32_t kValOff = kQueueOff + 16 * kQ * 2;
    constexpr int kCap = static_cast<int>((160 * 1024 - kValOff) / 8) - 1;
    constexpr int kCnt = static_cast<int>((160 * 1024 - kValOff) / 4);
    static_assert(kValOff % 16 == 0 && kCap > 0 && kMapOff < 65536, "LDS layout");
    constexpr uint32_t kLdsBytes = kAdj ? kValOff + kCnt * 4 : kValOff + (kCap + 1) * 8;
    __shared__ __attribute__((aligned(16))) uint8_t lds[kLdsBytes];
    uint32_t* bases = reinterpret_cast<uint32_t*>(lds);
    uint8_t* map = lds + kMapOff;
    double* vals = reinterpret_cast<double*>(lds + kValOff);
    uint32_t* cnt = reinterpret_cast<uint32_t*>(lds + kValOff);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    uint16_t* q = reinterpret_cast<uint16_t*>(lds + kQueueOff) + wv * kQ;
    const int G = a.G;
    const int64_t count = a.t_hi - a.t_lo;
    TailStats ts{};
    if constexpr (kAdj) ts = *adj.tail;

    // the (part, group) work list, part-major; workgroup b runs on XCD b % n_xcd,
    // and each XCD takes a contiguous share of the list
    const int64_t NGr = a.g_hi - a.g_lo;
    const int64_t n_items = static_cast<int64_t>(a.P) * NGr;
    const int64_t n_wg = gridDim.x;
    const int64_t per_x = n_wg / a.n_xcd;
    const int64_t l = static_cast<int64_t>(blockIdx.x % a.n_xcd) * per_x + blockIdx.x / a.n_xcd;
    int64_t it = l * n_items / n_wg;
    const int64_t it_end = (l + 1) * n_items / n_wg;

    // the backward's counters to W_mean once every wave is done with the part,
    // in the byte map's event order; the part before the first has none
    int prev_pq = -1;
    auto flush_counts = [&]() {
        __syncthreads();
        const int64_t ebase = static_cast<int64_t>(prev_pq) << kStreamShift;
        for (int e = threadIdx.x; e < kQSize; e += blockDim.x) {
            const uint32_t b = map[e];
            if (!b) continue;
            const uint32_t r = bases[e >> 7] + b;
            if (r >= static_cast<uint32_t>(kCnt)) continue;
            const uint32_t cv = cnt[r];
            if (cv) atomicAdd(reinterpret_cast<unsigned long long*>(&adj.w_mean[ebase + e]),
                              static_cast<unsigned long long>(cv));
        }
    };

    while (it < it_end) {
        if constexpr (kAdj) {
            if (prev_pq >= 0) flush_counts();
        }
        const int pq = static_cast<int>(it / NGr);
        const int64_t seg_end = min(it_end, static_cast<int64_t>(pq + 1) * NGr);
        const int64_t ga = a.g_lo + (it - static_cast<int64_t>(pq) * NGr);
        const int64_t gb = a.g_lo + (seg_end - static_cast<int64_t>(pq) * NGr);
        it = seg_end;
        // ---- the LDS image of stream part pq, from the part image of the
        // 2^18-event part that holds it
        const int ip = pq >> 2, is = pq & 3;
        const uint8_t* gimg = a.img + static_cast<int64_t>(ip) * kImgPartBytes;
        const uint64_t* gbm = reinterpret_cast<const uint64_t*>(gimg) + is * (kImgWords / 4);
        const uint16_t* gr16 = reinterpret_cast<const uint16_t*>(gimg + int64_t(kImgWords) * 8) + is * (kImgRank16 / 4);
        const uint32_t* gb32 = reinterpret_cast<const uint32_t*>(gimg + int64_t(kImgWords) * 8 + int64_t(kImgRank16) * 2) +
                               is * (kImgBase32 / 4);
        const uint32_t g0 = gb32[0];                // global rank of the part's first nonzero event
        // the part's nonzero count, from the rank of the next quarter's first
        // superblock (the next image part's, after the last quarter; unknown
        // after the catalogue's last image part): when every rank fits the LDS
        // copy of the values (the counters) the drain skips the L2 fallback
        // (the global atomics)
        const int64_t n_img = (a.C + (int64_t(1) << kImgShift) - 1) >> kImgShift;
        bool fits = false;
        if (is < 3 || ip + 1 < n_img) {
            const uint32_t g_next = is < 3 ? gb32[kImgBase32 / 4]
                                           : *reinterpret_cast<const uint32_t*>(
                                                 gimg + kImgPartBytes + int64_t(kImgWords) * 8 + int64_t(kImgRank16) * 2);
            fits = g_next - g0 <= static_cast<uint32_t>(kAdj ? kCnt : kCap);
        }
        __syncthreads();
        {
            // byte map: thread i covers events 64i .. 64i+63 (one bitmap word)
            const int i = threadIdx.x;
            const uint64_t w = gbm[i];
            uint32_t run = (i & 1) ? static_cast<uint32_t>(__popcll(gbm[i - 1])) : 0u;
            uint32_t* dst = reinterpret_cast<uint32_t*>(map + i * 64);
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                uint32_t pk = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const uint32_t bit = static_cast<uint32_t>(w >> (4 * k + b)) & 1u;
                    run += bit;
                    pk |= (bit ? run : 0u) << (8 * b);
                }
                dst[k] = pk;
            }
        }
        if (threadIdx.x < kQSize / 128) {
            const int k = threadIdx.x;
            bases[k] = gb32[k >> 5] + gr16[k] - g0 - 1u;
        }
        if constexpr (kAdj) {
            for (int k = threadIdx.x; k < kCnt; k += blockDim.x) cnt[k] = 0u;
        } else {
            for (int k = threadIdx.x; k <= kCap; k += blockDim.x) {
                const int64_t gk = static_cast<int64_t>(g0) + k;
                vals[k] = k < kCap && gk < a.C ? a.compact[gk] : 0.0;
            }
        }
        __syncthreads();

        // ---- this wave's groups [wa, wb) of the part
        const int64_t n = gb - ga;
        const int64_t wa = ga + wv * n / 16, wb = ga + (wv + 1) * n / 16;
        if constexpr (kAdj) prev_pq = pq;
        if (wa >= wb) continue;
        const uint16_t* ids = a.ids + a.part_base[pq];
        const uint32_t* gs = gstart_all + static_cast<int64_t>(pq) * (a.NG + 1);
        const uint16_t* ge = a.gend + static_cast<int64_t>(pq) * a.NG * kStreamGroupSlots;
        const double* gcompact = a.compact + g0;
        double* out_hi = a.part_hi + static_cast<int64_t>(pq) * count;
        float* out_lo = a.part_lo + static_cast<int64_t>(pq) * count;
        const int64_t ebase = static_cast<int64_t>(pq) << kStreamShift;   // catalogue ID of the part's event 0
        // B, lane i: where trial i of group g starts; lanes >= G: the group's
        // end.  The next group's trial ends are loaded with every batch (every
        // lane loads, lane 0 then drops its value; no value is carried over, so
        // no copy waits on the load) and added to its start when it begins.
        // The backward loads the next group's trial classes alongside.
        auto group_ends = [&](int64_t gg) -> uint32_t {
            return ge[gg * kStreamGroupSlots + (lane == 0 ? 0 : lane - 1)];
        };
        auto starts = [&](uint32_t s0, uint32_t ends) -> uint32_t { return lane == 0 ? s0 : s0 + ends; };
        auto group_class = [&](int64_t gg) -> uint32_t { return adj.cls[(gg - a.g_lo) * 64 + lane]; };
        // a group's IDs run from its start to the next group's start (its end
        // rounded up to the 8-ID chunk: the same chunks)
        int64_t g = wa;
        uint32_t rs = gs[g];
        uint32_t re = gs[g + 1];
        uint32_t B = starts(rs, group_ends(g));
        uint32_t next_ends = 0;
        uint32_t cls = 0, next_cls = 0;
        if constexpr (kAdj) cls = group_class(g);
        uint32_t c = rs;                            // first ID of the batch (a multiple of 8)
        int qs = kInf;                              // lane i: queue index of trial i's first hit
        int qn = 0;                                 // queue entries
        double acc_hi = 0.0, acc_lo = 0.0;
        double held_hi[kHeld];
        float held_lo[kHeld];
        int n_held = 0;

        auto load_batch = [&](uint32_t cb, uint32_t end, u32x4* v) {
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const uint32_t cu = cb + u * 64 * kChunkIds + lane * kChunkIds;
                const uint16_t* src = cu < end ? ids + cu : a.pad;
                v[u] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(src));
            }
        };
        // the batch after the one at c: the rest of this group, else the next group's first
        auto load_next = [&](u32x4* v) {
            next_ends = group_ends(g + 1 < wb ? g + 1 : g);
            if constexpr (kAdj) next_cls = group_class(g + 1 < wb ? g + 1 : g);
            if (c + kBatch < re) {
                load_batch(c + kBatch, re, v);
            } else {
                const bool more = g + 1 < wb;
                const uint32_t n_rs = more ? gs[g + 1] : 0u;
                const uint32_t n_re = more ? gs[g + 2] : 0u;
                load_batch(n_rs, n_re, v);
            }
        };
        // the queued hits: lane t takes trial t's entries, four at a time.
        // The loads of a step are issued together.
        auto rank = [&](uint32_t e) -> uint32_t {
            // rank among the part's nonzero events: the block's base (minus one)
            // plus the byte, which is 1 + the rank inside the block
            return bases[e >> 7] + map[e];
        };
        auto drain = [&]() {
            constexpr int kR = 4;
            int lo = __shfl(qs, lane), hi = __shfl(qs, (lane + 1) & 63);
            lo = lo < 0 ? 0 : (lo > qn ? qn : lo);
            hi = hi < 0 ? 0 : (hi > qn ? qn : hi);
            if (lane >= G) hi = lo;                 // lanes past the group's trials
            if constexpr (kAdj) {
                if (!(cls & 1u)) hi = lo;           // outside the aggregate band: no weight
                if (fits) {
                    // every rank has its LDS counter: whole steps unchecked,
                    // then the last one to three entries (their queue reads,
                    // at most two entries past a full queue, stay inside the
                    // allocation)
                    int j = lo;
                    for (; j + kR <= hi; j += kR) {
                        uint32_t e[kR], rk[kR];
#pragma unroll
                        for (int r2 = 0; r2 < kR; ++r2) e[r2] = q[j + r2];
#pragma unroll
                        for (int r2 = 0; r2 < kR; ++r2) rk[r2] = rank(e[r2]);
#pragma unroll
                        for (int r2 = 0; r2 < kR; ++r2) atomicAdd(&cnt[rk[r2]], 1u);
                    }
                    if (j < hi) {
                        uint32_t e[kR - 1], rk[kR - 1];
#pragma unroll
                        for (int r2 = 0; r2 < kR - 1; ++r2) e[r2] = q[j + r2];
#pragma unroll
                        for (int r2 = 0; r2 < kR - 1; ++r2) rk[r2] = rank(e[r2]);
#pragma unroll
                        for (int r2 = 0; r2 < kR - 1; ++r2)
                            if (j + r2 < hi) atomicAdd(&cnt[rk[r2]], 1u);
                    }
                } else {
                    for (int j = lo; j < hi; j += kR) {
                        uint32_t e[kR], rk[kR];
#pragma unroll
                        for (int r2 = 0; r2 < kR; ++r2) e[r2] = q[j + r2];
#pragma unroll
                        for (int r2 = 0; r2 < kR; ++r2) rk[r2] = rank(e[r2]);
#pragma unroll
                        for (int r2 = 0; r2 < kR; ++r2) {
                            if (j + r2 >= hi) continue;
                            if (rk[r2] < static_cast<uint32_t>(kCnt))
                                atomicAdd(&cnt[rk[r2]], 1u);
                            else
                                atomicAdd(reinterpret_cast<unsigned long long*>(&adj.w_mean[ebase + e[r2]]), 1ull);
                        }
                    }
                }
                if (cls & 6u) {
                    // a tail trial: its TVaR weight on each of its occurrences
                    const unsigned long long wt = static_cast<unsigned long long>((cls & 2u) ? ts.c_eq : ts.m - ts.c_gt);
                    for (int j = lo; j < hi; ++j)
                        atomicAdd(reinterpret_cast<unsigned long long*>(&adj.w_tvar[ebase + q[j]]), wt);
                }
            } else if (fits) {
                // every rank has its value in LDS: whole steps unchecked, then
                // the last one to three entries, whose idle slots read the 0.0
                // after the copied losses (their queue reads, at most two entries
                // past a full queue, stay inside the allocation)
                int j = lo;
                for (; j + kR <= hi; j += kR) {
                    uint32_t e[kR];
                    double v[kR];
#pragma unroll
                    for (int r2 = 0; r2 < kR; ++r2) e[r2] = q[j + r2];
#pragma unroll
                    for (int r2 = 0; r2 < kR; ++r2) v[r2] = vals[rank(e[r2])];
#pragma unroll
                    for (int r2 = 0; r2 < kR; ++r2) dd_add(acc_hi, acc_lo, v[r2]);
                }
                if (j < hi) {
                    uint32_t e[kR - 1];
                    double v[kR - 1];
#pragma unroll
                    for (int r2 = 0; r2 < kR - 1; ++r2) e[r2] = q[j + r2];
#pragma unroll
                    for (int r2 = 0; r2 < kR - 1; ++r2) v[r2] = vals[j + r2 < hi ? rank(e[r2]) : kCap];
#pragma unroll
                    for (int r2 = 0; r2 < kR - 1; ++r2) dd_add(acc_hi, acc_lo, v[r2]);
                }
            } else {
                for (int j = lo; j < hi; j += kR) {
                    // slots past the trial's last entry read whatever LDS follows
                    // (still inside the allocation), then the 0.0 after the copied
                    // losses, whose sum is exact
                    uint32_t e[kR], rk[kR];
                    bool valid[kR];
                    double v[kR];
#pragma unroll
                    for (int r2 = 0; r2 < kR; ++r2) {
                        valid[r2] = j + r2 < hi;
                        e[r2] = q[j + r2];
                    }
#pragma unroll
                    for (int r2 = 0; r2 < kR; ++r2) rk[r2] = rank(e[r2]);
                    // the LDS copy; ranks past it (parts with more nonzero losses
                    // than LDS holds) then read the value from L2
                    bool spill = false;
#pragma unroll
                    for (int r2 = 0; r2 < kR; ++r2) {
                        v[r2] = vals[valid[r2] ? min(rk[r2], static_cast<uint32_t>(kCap - 1)) : kCap];
                        spill |= valid[r2] && rk[r2] >= static_cast<uint32_t>(kCap);
                    }
                    if (__ballot(spill)) {
#pragma unroll
                        for (int r2 = 0; r2 < kR; ++r2)
                            if (valid[r2] && rk[r2] >= static_cast<uint32_t>(kCap)) v[r2] = gcompact[rk[r2]];
                    }
#pragma unroll
                    for (int r2 = 0; r2 < kR; ++r2) dd_add(acc_hi, acc_lo, v[r2]);
                }
            }
            qs = qs == kInf ? kInf : qs - qn;
            qn = 0;
            __builtin_amdgcn_wave_barrier();
        };
        // test a batch against the byte map, append its hits to the queue in
        // stream order, and note where each trial's hits start
        auto process = [&](const u32x4* v) {
            // Chunks past the group's end read padding or the next group's IDs;
            // their hits are queued after the group's end boundary (lanes >= G
            // note where it falls), so no trial takes them.
            uint32_t m[kU];                         // bit w: ID w of the lane's chunk is a hit
            bool hit[kU][8];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                uint32_t b[8];
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    b[2 * d] = map[v[u][d] & 0xFFFFu];
                    b[2 * d + 1] = map[v[u][d] >> 16];
                }
#pragma unroll
                for (int w = 0; w < 8; ++w) hit[u][w] = b[w] != 0;
                m[u] = lane_select<1>(hit[u][0]) | lane_select<2>(hit[u][1]) | lane_select<4>(hit[u][2]) |
                       lane_select<8>(hit[u][3]) | lane_select<16>(hit[u][4]) | lane_select<32>(hit[u][5]) |
                       lane_select<64>(hit[u][6]) | lane_select<128>(hit[u][7]);
            }
            // hit counts per chunk, prefix-summed over the wave two chunks at a time
            // (16-bit halves: at most 8 x 64 hits per load)
            uint32_t pre[kU], tot = 0, tot0 = 0;
            {
                const uint32_t ca = static_cast<uint32_t>(__popc(m[0]));
                const uint32_t cb = static_cast<uint32_t>(__popc(m[1]));
                const uint32_t sc = stream_wave_scan(ca | (cb << 16));
                const uint32_t tt = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(sc), 63));
                pre[0] = (sc & 0xFFFFu) - ca;
                pre[1] = (tt & 0xFFFFu) + (sc >> 16) - cb;
                tot0 = tt & 0xFFFFu;
                tot = tot0 + (tt >> 16);
            }
            // append the hits of load u; `skip` hits of the batch precede the queue's end
            auto append = [&](int u, uint32_t skip) {
                uint8_t* at = reinterpret_cast<uint8_t*>(q + qn + (pre[u] - skip));   // LDS byte address
#pragma unroll
                for (int w = 0; w < 8; ++w) {
                    if (hit[u][w]) *reinterpret_cast<uint16_t*>(at) = static_cast<uint16_t>(v[u][w >> 1] >> (16 * (w & 1)));
                    at += hit[u][w] ? 2 : 0;
                }
            };
            // trial starts at batch positions [from, to): the hits of the chunk
            // before the start's position, plus the chunk's queue offset
            const uint32_t rel = B - c;
            const uint32_t k = rel >> 3;
            const int src = static_cast<int>(k & 63u);
            const uint32_t p0 = static_cast<uint32_t>(__shfl(static_cast<int>((pre[0] << 8) | m[0]), src));
            const uint32_t p1 = static_cast<uint32_t>(__shfl(static_cast<int>((pre[1] << 8) | m[1]), src));
            const uint32_t pk = (k >> 6) == 0 ? p0 : p1;
            const int before = static_cast<int>(pk >> 8) + __popc((pk & 0xFFu) & ((1u << (rel & 7u)) - 1u));
            auto record = [&](uint32_t from, uint32_t to, int skip) {
                if (B >= c && rel >= from && rel < to) qs = qn + before - skip;
            };
            if (qn + static_cast<int>(tot) > kQ) drain();
            if (tot <= static_cast<uint32_t>(kQ)) {
                append(0, 0u);
                append(1, 0u);
                record(0u, kBatch, 0);
                qn += static_cast<int>(tot);
            } else {
                // more hits than the queue holds (dense layers): the first load's
                // hits, a drain, then the second load's (each fits an empty queue)
                const uint32_t t0 = tot0;
                append(0, 0u);
                record(0u, kBatch / 2, 0);
                qn += static_cast<int>(t0);
                drain();
                append(1, t0);
                record(kBatch / 2, kBatch, static_cast<int>(t0));
                qn += static_cast<int>(tot - t0);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };
        // Partial sums of the last kHeld groups wait in registers and are stored
        // together, then waited for at once: a store pending at the next wait
        // for a batch would make that wait cover every load in flight (stores
        // and loads share one counter and complete in either order), which at
        // every group's end would stall the stream
        auto flush = [&]() {
#pragma unroll
            for (int k = 0; k < kHeld; ++k) {
                const int64_t t = (g - k) * G + lane;
                if (k < n_held && lane < G && t >= a.t_lo && t < a.t_hi) {
                    out_hi[t - a.t_lo] = held_hi[k];
                    out_lo[t - a.t_lo] = held_lo[k];
                }
            }
            n_held = 0;
            __builtin_amdgcn_s_waitcnt(kWaitVm0);
        };
        // after a batch: advance; at the end of the group drain the queue, hold
        // the partial sums (the forward) and move to the next group (its first
        // batch is in flight).  Returns false after the wave's last group.
        auto step = [&]() -> bool {
            c += kBatch;
            if (c < re) return true;
            drain();
            if constexpr (!kAdj) {
                // the group's sums join the held results (newest first)
#pragma unroll
                for (int k = kHeld - 1; k > 0; --k) {
                    held_hi[k] = held_hi[k - 1];
                    held_lo[k] = held_lo[k - 1];
                }
                held_hi[0] = acc_hi + acc_lo;          // renormalised: |lo| <= ulp(hi) / 2
                held_lo[0] = static_cast<float>(acc_lo - (held_hi[0] - acc_hi));
                ++n_held;
                if (n_held == kHeld || g + 1 >= wb) flush();
                acc_hi = 0.0;
                acc_lo = 0.0;
            }
            qs = kInf;
            if (g + 1 >= wb) return false;
            ++g;
            rs = gs[g];
            re = gs[g + 1];
            B = starts(rs, next_ends);
            if constexpr (kAdj) cls = next_cls;
            c = rs;
            return true;
        };

        // two register buffers in turn, so the next batch's loads stay in
        // flight while this one is tested
        u32x4 bufA[kU], bufB[kU];
        load_batch(c, re, bufA);
        for (;;) {
            load_next(bufB);
            process(bufA);
            if (!step()) break;
            load_next(bufA);
            process(bufB);
            if (!step()) break;
        }
    }
    if constexpr (kAdj) {
        if (prev_pq >= 0) flush_counts();
    }
}

// the trial classes of StreamAdjArgs, one byte per (group, lane) slot
__global__ __launch_bounds__(256) void stream_class_kernel(const double* __restrict__ S, const double* __restrict__ ylt,
                                                           const TailStats* __restrict__ tail, double aggR, double aggL,
                                                           int64_t t_lo, int64_t t_hi, int G, int64_t g_lo,
                                                           int64_t n_slots, uint8_t* __restrict__ cls) {
    const TailStats ts = *tail;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n_slots; i += stride) {
        const int lane = static_cast<int>(i & 63);
        const int64_t t = (g_lo + (i >> 6)) * G + lane;
        uint32_t c = 0;
        if (lane < G && t >= t_lo && t < t_hi) {
            const int64_t k = t - t_lo;
            const double ta = S[k] - aggR;
            if ((ta > 0.0) && (ta < aggL)) {
                // year losses are >= 0, so their bit patterns order like their values
                const uint64_t key = __double_as_longlong(ylt[k] + 0.0);
                c = 1u | (key > ts.v_bits ? 2u : (key == ts.v_bits ? 4u : 0u));
            }
        }
        cls[i] = static_cast<uint8_t>(c);
    }
}

__global__ __launch_bounds__(256) void stream_combine_kernel(const double* __restrict__ part_hi,
                                                             const float* __restrict__ part_lo, int P, int64_t count,
                                                             double aggR, double aggL,
                                                             const LayerArgs* __restrict__ L_dev,
                                                             double* __restrict__ ylt, double* __restrict__ S_out) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= count) return;
    if (L_dev) {                                    // terms from device memory (graph replays)
        aggR = L_dev->aggR;
        aggL = L_dev->aggL;
    }
    double hi = 0.0, lo = 0.0;
    for (int p = 0; p < P; ++p)
        dd_merge(hi, lo, part_hi[p * count + k], static_cast<double>(part_lo[p * count + k]));
    const double S = hi + lo;
    ylt[k] = apply_terms(S, aggR, aggL);
    if (S_out) S_out[k] = S;
}

// trials per group: enough that the group's IDs fill whole batches of
// 512-ID loads with little left over, given the mean IDs per (trial, part)
int choose_group_trials(double lam) {
    int best_g = kStreamGroupMax;
    double best = 1e300;
    for (int g = kStreamGroupMax; g >= 16; --g) {
        const double mean = g * lam, sd = std::sqrt(mean > 0.0 ? mean : 0.0);
        const double chunks = (mean + 2.5 * sd) / kChunkIds + 1.0;
        const double loads = std::ceil(chunks / 64.0);
        const double cost = (loads * 512.0 * 5.0 + 200.0) / g;
        if (cost < best - 1e-9) {
            best = cost;
            best_g = g;
        }
    }
    return best_g;
}

}  // namespace

hipError_t build_stream_layout(const int64_t* offsets, const uint32_t* ids, int64_t N, int64_t n_events, int64_t C,
                               int n_cu, hipStream_t s, StreamLayout* out) {
    *out = StreamLayout{};
    const int P = static_cast<int>((C + kQSize - 1) / kQSize);
    if (N < 1 || P < 1 || P > kMaxStreamParts) return hipSuccess;      // layout not used
    const int G = choose_group_trials(static_cast<double>(n_events) / (static_cast<double>(N) * P));
    const int64_t NG = (N + G - 1) / G;
    const int64_t n_grp = static_cast<int64_t>(P) * NG;
    hipError_t e;
    int32_t* cnt = nullptr;
    uint32_t* gsize = nullptr;
    uint64_t* plen = nullptr;
    uint32_t* flag = nullptr;
    std::vector<uint64_t> h_len(P);
    std::vector<int64_t> h_base(P + 1);
    uint32_t h_flag = 0;
    int64_t blocks = (N + 3) / 4;
    if (blocks > int64_t(n_cu) * 16) blocks = int64_t(n_cu) * 16;
    if ((e = dev_alloc(reinterpret_cast<void**>(&cnt), sizeof(int32_t) * N * P, s)) != hipSuccess) goto fail;
    if ((e = dev_alloc(reinterpret_cast<void**>(&gsize), sizeof(uint32_t) * n_grp, s)) != hipSuccess) goto fail;
    if ((e = dev_alloc(reinterpret_cast<void**>(&plen), sizeof(uint64_t) * P, s)) != hipSuccess) goto fail;
    if ((e = dev_alloc(reinterpret_cast<void**>(&flag), sizeof(uint32_t), s)) != hipSuccess) goto fail;
    if ((e = dev_alloc(reinterpret_cast<void**>(&out->gend), sizeof(uint16_t) * n_grp * kStreamGroupSlots, s)) !=
        hipSuccess)
        goto fail;
    if ((e = dev_alloc(reinterpret_cast<void**>(&out->gstart), sizeof(uint32_t) * P * (NG + 1), s)) != hipSuccess)
        goto fail;
    if ((e = dev_alloc(reinterpret_cast<void**>(&out->part_base), sizeof(int64_t) * (P + 1), s)) != hipSuccess)
        goto fail;
    if ((e = hipMemsetAsync(flag, 0, sizeof(uint32_t), s)) != hipSuccess) goto fail;
    hipLaunchKernelGGL(stream_count_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, offsets, ids, N, P,
                       cnt);
    if ((e = hipGetLastError()) != hipSuccess) goto fail;
    hipLaunchKernelGGL(stream_group_kernel, dim3(static_cast<uint32_t>((n_grp + 255) / 256)), dim3(256), 0, s, cnt, N,
                       P, G, NG, out->gend, gsize, flag);
    if ((e = hipGetLastError()) != hipSuccess) goto fail;
    hipLaunchKernelGGL(stream_scan_kernel, dim3(static_cast<uint32_t>(P)), dim3(1024), 0, s, gsize, NG, out->gstart,
                       plen, flag);
    if ((e = hipGetLastError()) != hipSuccess) goto fail;
    if ((e = hipMemcpyAsync(h_len.data(), plen, sizeof(uint64_t) * P, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(&h_flag, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        goto fail;
    if (h_flag) {                       // a group or a part too large for 16/32-bit offsets: not used
        e = hipSuccess;
        goto fail;
    }
    h_base[0] = 0;
    for (int q = 0; q < P; ++q) h_base[q + 1] = h_base[q] + static_cast<int64_t>(h_len[q]);
    out->length = h_base[P];
    if ((e = hipMemcpyAsync(out->part_base, h_base.data(), sizeof(int64_t) * (P + 1), hipMemcpyHostToDevice, s)) !=
        hipSuccess)
        goto fail;
    if ((e = dev_alloc(reinterpret_cast<void**>(&out->ids), sizeof(uint16_t) * (out->length + kStreamPad), s)) !=
        hipSuccess)
        goto fail;
    {
        const int64_t n32 = (out->length + kStreamPad) / 2;
        int64_t fb = (n32 + 255) / 256;
        if (fb > 8192) fb = 8192;
        hipLaunchKernelGGL(stream_fill_kernel, dim3(static_cast<uint32_t>(fb)), dim3(256), 0, s,
                           reinterpret_cast<uint32_t*>(out->ids), n32, 0xFFFFFFFFu);
        if ((e = hipGetLastError()) != hipSuccess) goto fail;
    }
    {
        int64_t gb = NG;
        if (gb > int64_t(n_cu)) gb = n_cu;                 // one 16-wave workgroup per CU (the stage fills LDS)
        hipLaunchKernelGGL(stream_group_scatter_kernel, dim3(static_cast<uint32_t>(gb)), dim3(1024), 0, s, offsets,
                           ids, N, P, G, NG, out->part_base, out->gstart, out->gend, out->ids);
    }
    if ((e = hipGetLastError()) != hipSuccess) goto fail;
    // temporaries go back to the library's device memory cache: no free waits for the device
    dev_free(cnt, s);
    dev_free(gsize, s);
    dev_free(plen, s);
    dev_free(flag, s);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) {
        free_stream_layout(out, s);
        return e;
    }
    out->P = P;
    out->G = G;
    out->NG = NG;
    out->bytes = static_cast<int64_t>(sizeof(uint16_t)) * (out->length + kStreamPad) +
                 static_cast<int64_t>(sizeof(uint16_t)) * n_grp * kStreamGroupSlots +
                 static_cast<int64_t>(sizeof(uint32_t)) * P * (NG + 1) + static_cast<int64_t>(sizeof(int64_t)) * (P + 1);
    return hipSuccess;
fail:
    if (cnt) dev_free(cnt, s);
    if (gsize) dev_free(gsize, s);
    if (plen) dev_free(plen, s);
    if (flag) dev_free(flag, s);
    free_stream_layout(out, s);
    (void)hipStreamSynchronize(s);
    return e;
}

void free_stream_layout(StreamLayout* L, hipStream_t s) {
    if (L->ids) dev_free(L->ids, s);
    if (L->part_base) dev_free(L->part_base, s);
    if (L->gstart) dev_free(L->gstart, s);
    if (L->gend) dev_free(L->gend, s);
    *L = StreamLayout{};
}

int64_t stream_partials_bytes(const StreamLayout& lay, int64_t trials) {
    const int64_t n = static_cast<int64_t>(lay.P) * (trials > 0 ? trials : 1);
    return static_cast<int64_t>(sizeof(double) + sizeof(float)) * n + 256;
}

namespace {

StreamPassArgs pass_args(const StreamLayout& lay, int64_t C, const LayerArgs& L, void* part_scratch, int n_img_parts) {
    StreamPassArgs a{};
    a.ids = lay.ids;
    a.part_base = lay.part_base;
    a.gstart = lay.gstart;
    a.gend = lay.gend;
    a.img = static_cast<const uint8_t*>(part_scratch);
    a.compact = part_compact_values(part_scratch, n_img_parts);
    a.C = C;
    a.P = lay.P;
    a.G = lay.G;
    a.NG = lay.NG;
    a.t_lo = L.trial_begin;
    a.t_hi = L.trial_begin + L.trial_count;
    a.g_lo = a.t_lo / lay.G;
    a.g_hi = (a.t_hi + lay.G - 1) / lay.G;
    a.pad = lay.ids + lay.length;
    a.n_xcd = kXcds;
    return a;
}

// one 1024-thread workgroup per CU (its LDS holds the part's byte map and
// values or counters), a multiple of the XCD count
uint32_t pass_grid(int n_cu) {
    int64_t grid = int64_t(n_cu);
    grid -= grid % kXcds;
    if (grid < kXcds) grid = kXcds;
    return static_cast<uint32_t>(grid);
}

}  // namespace

hipError_t launch_stream_pass(const StreamLayout& lay, int64_t C, const LayerArgs& L, void* part_scratch,
                              int n_img_parts, void* partials, int n_cu, hipStream_t s) {
    if (L.trial_count <= 0) return hipSuccess;
    if (lay.P <= 0 || (lay.P - 1) / 4 >= n_img_parts) return hipErrorInvalidValue;
    StreamPassArgs a = pass_args(lay, C, L, part_scratch, n_img_parts);
    a.part_hi = static_cast<double*>(partials);
    a.part_lo = reinterpret_cast<float*>(a.part_hi + static_cast<int64_t>(lay.P) * L.trial_count);
    hipLaunchKernelGGL(stream_pass_kernel<false>, dim3(pass_grid(n_cu)), dim3(1024), 0, s, a, StreamAdjArgs{},
                       a.gstart);
    return hipGetLastError();
}

int64_t stream_adjoint_scratch_bytes(int64_t trials) {
    // (group, lane) class slots: at most trials / 16 + 2 groups of 64
    return 4 * (trials > 0 ? trials : 0) + 256;
}

hipError_t launch_stream_adjoint(const StreamLayout& lay, int64_t C, const LayerArgs& L, void* part_scratch,
                                 int n_img_parts, const double* S, const double* ylt, const TailStats* tail,
                                 void* scratch, int64_t scratch_bytes, uint64_t* w_mean, uint64_t* w_tvar, int n_cu,
                                 hipStream_t s) {
    if (L.trial_count <= 0) return hipSuccess;
    if (lay.P <= 0 || (lay.P - 1) / 4 >= n_img_parts) return hipErrorInvalidValue;
    const StreamPassArgs a = pass_args(lay, C, L, part_scratch, n_img_parts);
    const int64_t n_slots = (a.g_hi - a.g_lo) * 64;
    if (n_slots > scratch_bytes) return hipErrorInvalidValue;
    StreamAdjArgs adj{};
    adj.cls = static_cast<const uint8_t*>(scratch);
    adj.w_mean = w_mean;
    adj.w_tvar = w_tvar;
    adj.tail = tail;
    int64_t cb = (n_slots + 255) / 256;
    if (cb > int64_t(n_cu) * 8) cb = int64_t(n_cu) * 8;
    hipLaunchKernelGGL(stream_class_kernel, dim3(static_cast<uint32_t>(cb)), dim3(256), 0, s, S, ylt, tail, L.aggR,
                       L.aggL, a.t_lo, a.t_hi, a.G, a.g_lo, n_slots, static_cast<uint8_t*>(scratch));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(stream_pass_kernel<true>, dim3(pass_grid(n_cu)), dim3(1024), 0, s, a, adj, a.gstart);
    return hipGetLastError();
}

hipError_t launch_stream_combine(const StreamLayout& lay, const LayerArgs& L, const LayerArgs* L_dev,
                                 const void* partials, double* ylt, double* S, hipStream_t s) {
    if (L.trial_count <= 0) return hipSuccess;
    const double* hi = static_cast<const double*>(partials);
    const float* lo = reinterpret_cast<const float*>(hi + static_cast<int64_t>(lay.P) * L.trial_count);
    const int64_t blocks = (L.trial_count + 255) / 256;
    hipLaunchKernelGGL(stream_combine_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, hi, lo, lay.P,
                       L.trial_count, L.aggR, L.aggL, L_dev, ylt, S);
    return hipGetLastError();
}

}  // namespace ara
