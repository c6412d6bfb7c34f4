// Catalogue-partitioned trial pass.
//
// Random 8-byte gathers from a table larger than L2 run an order of magnitude
// below the HBM stream rate on gfx950, and most occurrences of a layer carry
// zero loss (an event absent from every ELT of the layer, or below the
// occurrence retention).  So the per-event question "is o(E) nonzero, and
// where is its value" is answered from LDS:
//
//  * the catalogue is cut into parts of 2^18 events; for each part the fold
//    builds a 37,120-byte image: a 32 KB bitmap of nonzero o(E), a 16-bit rank
//    per 128 events relative to its 4096-event superblock, and the global rank
//    of each superblock; the nonzero values themselves go, in catalogue order,
//    to a compact array small enough to stay in L2;
//  * at table creation the YET is laid out part-major inside tiles of
//    consecutive trials (tile -> part -> trial -> that trial's events of that
//    part in time order, each segment padded to 16 bytes with an ID no event
//    has), so a workgroup can hold one part image in LDS and stream exactly
//    the events that need it;
//  * a workgroup takes a tile, walks the parts in order, and for each trial
//    adds the part's partial sum (double-double) into the trial's LDS
//    accumulator; the trial's owner and the part order are fixed, so the
//    result does not depend on scheduling.
#include <vector>

#include <type_traits>

#include "ara_internal.hpp"

namespace ara {

namespace {

constexpr int kPartShift = 18;
constexpr int64_t kPartSize = int64_t(1) << kPartShift;       // catalogue events per part
constexpr int kWords = kPartSize / 64;                        // 4096 u64 bitmap words
constexpr int kRank16 = kPartSize / 128;                      // 2048 u16
constexpr int kSuperShift = 12;
constexpr int kSuper = 1 << kSuperShift;                      // 4096 events per superblock
constexpr int kBase32 = kPartSize / kSuper;                   // 64 u32
constexpr int64_t kImgBytes = int64_t(kWords) * 8 + int64_t(kRank16) * 2 + int64_t(kBase32) * 4;
static_assert(kImgBytes == 37120 && kImgBytes == kImgPartBytes && kPartShift == kImgShift, "part image layout");
static_assert(kImgBytes % 16 == 0, "16-byte copies");
constexpr int kTileMax = 256;                                 // trials per tile (LDS accumulators)
constexpr int kTileAlign = 32;                                // tiles start on 128-byte boundaries
constexpr uint32_t kSentinel = 0xFFFFFFFFu;

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// ---------------------------------------------------------------------------
// create-time layout
// ---------------------------------------------------------------------------

// events per (trial, part), one wavefront per trial
__global__ __launch_bounds__(256) void part_count_kernel(const int64_t* __restrict__ offsets,
                                                         const uint32_t* __restrict__ ids, int64_t N, int P,
                                                         int32_t* __restrict__ cnt) {
    __shared__ int32_t c[4][kMaxParts];
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
                    if (c0 + k * 64 + lane < e) atomicAdd(&c[w][idk[k] >> kPartShift], 1);
            }
        }
        __builtin_amdgcn_wave_barrier();
        for (int p = lane; p < P; p += 64) cnt[t * P + p] = c[w][p];
        __builtin_amdgcn_wave_barrier();
    }
}

// per tile: layout-order exclusive scan of the padded segment sizes
__global__ __launch_bounds__(256) void tile_scan_kernel(const int32_t* __restrict__ cnt, int64_t N, int P, int T,
                                                        uint32_t* __restrict__ seg_rel, int64_t* __restrict__ tile_size) {
    __shared__ int64_t part_sum[256];
    const int64_t tile = blockIdx.x;
    const int64_t t0 = tile * T;
    const int Tk = static_cast<int>(N - t0 < T ? N - t0 : T);
    const int n = P * Tk;
    const int64_t base = tile * (static_cast<int64_t>(T) * P + 1);
    const int per = (n + 255) / 256;
    const int j0 = threadIdx.x * per;
    int64_t local = 0;
    for (int j = j0; j < j0 + per && j < n; ++j) {
        const int p = j / Tk, i = j % Tk;
        local += (cnt[(t0 + i) * P + p] + 3) & ~3;
    }
    part_sum[threadIdx.x] = local;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        int64_t add = threadIdx.x >= off ? part_sum[threadIdx.x - off] : 0;
        __syncthreads();
        part_sum[threadIdx.x] += add;
        __syncthreads();
    }
    int64_t run = part_sum[threadIdx.x] - local;
    for (int j = j0; j < j0 + per && j < n; ++j) {
        const int p = j / Tk, i = j % Tk;
        seg_rel[base + j] = static_cast<uint32_t>(run);
        run += (cnt[(t0 + i) * P + p] + 3) & ~3;
    }
    if (threadIdx.x == 255) {
        seg_rel[base + n] = static_cast<uint32_t>(part_sum[255]);
        tile_size[tile] = part_sum[255];
    }
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Scatter of each trial's IDs into its per-part segments of the tiled copy,
// one workgroup per run of kChunkTrials trials of a tile.  Inside a tile each
// part's segments of consecutive trials are consecutive, so the run's
// segments of every part form one contiguous range per part: they are staged
// in LDS (part after part, the padding that ends each trial's segment filled
// with the sentinel), the trials scattered there one wave per trial,
// and each part's range then leaves in coalesced 4-byte stores instead of
// writes spread over up to P lines per 64 IDs.  Per 64 IDs the lanes holding
// an ID of this lane's part are the AND, over the part number's bits, of that
// bit's ballot or its complement; a lane's rank among the earlier ones places
// it, all 64 write in one store, and the last lane of each part moves its
// cursor on.  A run whose IDs exceed the stage is scattered straight to the
// copy.
constexpr int kChunkTrials = 32;
constexpr int kPartStageIds = 36 * 1024;        // 144 KB of LDS
__global__ __launch_bounds__(1024) void part_scatter_kernel(const int64_t* __restrict__ offsets,
                                                            const uint32_t* __restrict__ ids, int64_t N, int P, int T,
                                                            const uint32_t* __restrict__ seg_rel,
                                                            const int64_t* __restrict__ tile_start,
                                                            uint32_t* __restrict__ pids) {
    __shared__ uint32_t stage[kPartStageIds];
    __shared__ uint32_t sseg[kMaxParts + 1];          // staged start of each part's range
    __shared__ int64_t cur[16][kMaxParts];
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int n_bits = P > 1 ? 32 - __builtin_clz(static_cast<uint32_t>(P - 1)) : 0;
    const uint64_t above = lane == 63 ? 0ull : (~0ull << (lane + 1));
    const int64_t n_tiles = (N + T - 1) / T;
    const int64_t per_tile = (T + kChunkTrials - 1) / kChunkTrials;
    for (int64_t r = blockIdx.x; r < n_tiles * per_tile; r += gridDim.x) {
        const int64_t tile = r / per_tile;
        const int64_t t0 = tile * T;
        const int Tk = static_cast<int>(N - t0 < T ? N - t0 : T);
        const int i0 = static_cast<int>(r - tile * per_tile) * kChunkTrials;
        if (i0 >= Tk) continue;                                   // uniform over the workgroup
        const int i1 = i0 + kChunkTrials < Tk ? i0 + kChunkTrials : Tk;
        const int64_t base = tile * (static_cast<int64_t>(T) * P + 1);
        if (w == 0) {                                  // each part's range size, scanned over the wave
            uint32_t n = 0;
            if (lane < P)
                n = seg_rel[base + static_cast<int64_t>(lane) * Tk + i1] - seg_rel[base + static_cast<int64_t>(lane) * Tk + i0];
            uint32_t inc = n;
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t v = __shfl_up(inc, off, 64);
                if (lane >= off) inc += v;
            }
            if (lane < P) sseg[lane] = inc - n;
            if (lane == P - 1) sseg[P] = inc;
        }
        __syncthreads();
        const bool staged = sseg[P] <= static_cast<uint32_t>(kPartStageIds);
        if (staged) {                                  // segments end in sentinel padding, as in the copy
            for (uint32_t u = threadIdx.x; u < sseg[P]; u += blockDim.x) stage[u] = kSentinel;
        }
        __syncthreads();
        for (int i = i0 + w; i < i1; i += 16) {
            const int64_t t = t0 + i;
            for (int p = lane; p < P; p += 64) {
                const int64_t k = base + static_cast<int64_t>(p) * Tk;
                cur[w][p] = staged ? sseg[p] + (seg_rel[k + i] - seg_rel[k + i0]) : tile_start[tile] + seg_rel[k + i];
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
                    const int pid = static_cast<int>(id >> kPartShift);
                    uint64_t same = __ballot(valid);
                    for (int bit = 0; bit < n_bits; ++bit) {
                        const bool set = ((pid >> bit) & 1) != 0;
                        const uint64_t lanes = __ballot(set);
                        same &= set ? lanes : ~lanes;
                    }
                    const int64_t at = cur[w][pid];
                    if (valid) {
                        const int64_t to = at + __popcll(same & lanemask_lt());
                        if (staged)
                            stage[to] = id;
                        else
                            pids[to] = id;
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
            for (int p = w; p < P; p += 16) {
                const int64_t k = base + static_cast<int64_t>(p) * Tk;
                uint32_t* dst = pids + tile_start[tile] + seg_rel[k + i0];
                const uint32_t s0 = sseg[p], n = sseg[p + 1] - s0;
                for (uint32_t u = lane; u < n; u += 64) dst[u] = stage[s0 + u];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// per-request part images
// ---------------------------------------------------------------------------

// one workgroup (256 threads) per superblock of 4096 catalogue events:
// bitmap words, per-128 ranks inside the superblock, superblock count
__global__ __launch_bounds__(256) void part_image_kernel(const double* __restrict__ o, int64_t C,
                                                         uint8_t* __restrict__ img, uint32_t* __restrict__ sb_count,
                                                         int64_t o_stride, int64_t img_stride, int64_t sb_stride) {
    __shared__ uint32_t wc[64];
    o += blockIdx.y * o_stride;
    img += blockIdx.y * img_stride;
    sb_count += blockIdx.y * sb_stride;
    const int64_t sb = blockIdx.x;
    const int64_t e0 = sb * kSuper;
    const int64_t part = e0 >> kPartShift;
    const int ls = static_cast<int>((e0 & (kPartSize - 1)) >> kSuperShift);
    uint64_t* bm = reinterpret_cast<uint64_t*>(img + part * kImgBytes);
    uint16_t* r16 = reinterpret_cast<uint16_t*>(img + part * kImgBytes + int64_t(kWords) * 8);
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    for (int k = 0; k < 16; ++k) {
        const int word = w * 16 + k;                       // 0..63 inside the superblock
        const int64_t E = e0 + word * 64 + lane;
        const bool nz = E < C && o[E] != 0.0;
        const uint64_t bits = __ballot(nz);
        if (lane == 0) {
            bm[ls * 64 + word] = bits;
            wc[word] = __popcll(bits);
        }
    }
    __syncthreads();
    if (threadIdx.x < 32) {
        uint32_t before = 0;
        for (int b = 0; b < static_cast<int>(threadIdx.x); ++b) before += wc[2 * b] + wc[2 * b + 1];
        r16[ls * 32 + threadIdx.x] = static_cast<uint16_t>(before);
    }
    if (threadIdx.x == 0) {
        uint32_t total = 0;
        for (int k = 0; k < 64; ++k) total += wc[k];
        sb_count[sb] = total;
    }
}

// The fold and the part images in one pass: one workgroup (256 threads) per
// superblock of 4096 catalogue events.  The superblock's ELT-combined losses
// y are summed in LDS from the sparse pool: for each ELT of the layer, in
// layer order, the chunk's nonzero entries (distinct events) each add their
// per-ELT net loss, with a barrier between ELTs.  An absent loss adds +0.0
// (retentions are >= 0), which leaves y unchanged, so y is bit-identical to
// summing every ELT's dense row in layer order.  The entries of all the
// layer's ELTs are first copied to LDS with independent loads (up to kStage
// of them; the rest are read in place), so the ELTs cost one load latency,
// not one each.  Then o, the bitmap words, the per-128 ranks and the
// superblock count are written, and the superblock's nonzero o, packed in
// event order, go to its 4096-value slot of `stage` (compact_stage_kernel
// moves them to their global ranks).
__device__ __forceinline__ void fold_image_body(const SparsePool& sp, int64_t C, const LayerArgs& L,
                                                double* __restrict__ o, uint8_t* __restrict__ img,
                                                uint32_t* __restrict__ sb_count, double* __restrict__ stage) {
    constexpr int kStage = 2048;                    // entries staged in LDS
    __shared__ uint32_t wc[64];
    __shared__ double ys[kSuper];
    __shared__ double sval[kStage];
    __shared__ uint16_t sev[kStage];
    __shared__ int64_t gstart[kMaxJ];               // ELT j's first entry of this chunk in the pool
    __shared__ int32_t fpre[kMaxJ + 1];             // ELT j's entries are [fpre[j], fpre[j+1]) of the chunk's list
    const int64_t sb = blockIdx.x;
    const int64_t e0 = sb * kSuper;
    const int64_t part = e0 >> kPartShift;
    const int ls = static_cast<int>((e0 & (kPartSize - 1)) >> kSuperShift);
    uint64_t* bm = reinterpret_cast<uint64_t*>(img + part * kImgBytes);
    uint16_t* r16 = reinterpret_cast<uint16_t*>(img + part * kImgBytes + int64_t(kWords) * 8);
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < kSuper; i += blockDim.x) ys[i] = 0.0;
    const int J = sb < sp.n_chunks ? L.J : 0;       // J <= kMaxJ <= 64: one wave holds the ELTs
    if (w == 0) {
        int32_t cnt = 0;
        if (lane < J) {
            const int64_t key = static_cast<int64_t>(L.idx[lane]) * sp.n_chunks + sb;
            const int64_t b = sp.chunk_off[key];
            gstart[lane] = b;
            cnt = static_cast<int32_t>(sp.chunk_off[key + 1] - b);    // <= 4096
        }
        int32_t inc = cnt;                          // inclusive scan over the wave
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t v = __shfl_up(inc, off, kWave);
            if (lane >= off) inc += v;
        }
        if (lane < J) fpre[lane + 1] = inc;
        if (lane == 0) fpre[0] = 0;
    }
    __syncthreads();
    const int n_list = fpre[J];
    const int staged = n_list < kStage ? n_list : kStage;
    // ELT of entry f of the list: the first j whose range ends past f
    auto elt_of = [&](int f) {
        int lo = 0, hi = J - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (fpre[mid + 1] > f) hi = mid;
            else lo = mid + 1;
        }
        return lo;
    };
    for (int f0 = threadIdx.x; f0 < staged; f0 += 4 * blockDim.x) {
        uint16_t ev[4];
        double val[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int f = f0 + u * static_cast<int>(blockDim.x);
            if (f < staged) {
                const int j = elt_of(f);
                const int64_t k = gstart[j] + (f - fpre[j]);
                ev[u] = sp.ev[k];
                val[u] = sp.val[k];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int f = f0 + u * static_cast<int>(blockDim.x);
            if (f < staged) {
                sev[f] = ev[u];
                sval[f] = val[u];
            }
        }
    }
    __syncthreads();
    for (int j = 0; j < J; ++j) {
        const double R = L.R[j], Lim = L.Lim[j];
        const int fe = fpre[j + 1];
        for (int f = fpre[j] + static_cast<int>(threadIdx.x); f < fe; f += blockDim.x) {
            int ev;
            double v;
            if (f < kStage) {
                ev = sev[f];
                v = sval[f];
            } else {
                const int64_t k = gstart[j] + (f - fpre[j]);
                ev = sp.ev[k];
                v = sp.val[k];
            }
            ys[ev] = ys[ev] + apply_terms(v, R, Lim);
        }
        __syncthreads();
    }
    const int64_t eb = e0 + static_cast<int64_t>(w) * 16 * 64 + lane;   // event of word 0 of this wave
    double vk[16];
    uint64_t bk[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int word = w * 16 + k;
        const int64_t E = eb + k * 64;
        const double v = apply_terms(ys[word * 64 + lane], L.occR, L.occL);
        if (E < C) o[E] = v;
        const uint64_t bits = __ballot(E < C && v != 0.0);
        vk[k] = v;
        bk[k] = bits;
        if (lane == 0) {
            bm[ls * 64 + word] = bits;
            wc[word] = __popcll(bits);
        }
    }
    __syncthreads();
    {   // the nonzero o packed in event order: the wave's first word starts
        // after the counts of the words before it
        uint32_t at = 0;
        for (int k = 0; k < w * 16; ++k) at += wc[k];
        double* dst = stage + sb * kSuper;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if ((bk[k] >> lane) & 1ull) dst[at + __popcll(bk[k] & lanemask_lt())] = vk[k];
            at += __popcll(bk[k]);
        }
    }
    if (threadIdx.x < 32) {
        uint32_t before = 0;
        for (int b = 0; b < static_cast<int>(threadIdx.x); ++b) before += wc[2 * b] + wc[2 * b + 1];
        r16[ls * 32 + threadIdx.x] = static_cast<uint16_t>(before);
    }
    if (threadIdx.x == 0) {
        uint32_t total = 0;
        for (int k = 0; k < 64; ++k) total += wc[k];
        sb_count[sb] = total;
    }
}

// terms as kernel arguments (eager runs) or read from device memory (graph
// replays, whose terms may change between replays)
__global__ __launch_bounds__(256) void fold_image_kernel(SparsePool sp, int64_t C, LayerArgs L,
                                                         double* __restrict__ o, uint8_t* __restrict__ img,
                                                         uint32_t* __restrict__ sb_count, double* __restrict__ stage) {
    fold_image_body(sp, C, L, o, img, sb_count, stage);
}
__global__ __launch_bounds__(256) void fold_image_dev_kernel(SparsePool sp, int64_t C,
                                                             const LayerArgs* __restrict__ L, double* __restrict__ o,
                                                             uint8_t* __restrict__ img, uint32_t* __restrict__ sb_count,
                                                             double* __restrict__ stage) {
    fold_image_body(sp, C, *L, o, img, sb_count, stage);
}

// After the fold: each superblock's global rank (the nonzero count of the
// superblocks before it, summed by its own workgroup) goes to its part's base
// table, and its packed nonzero o to compact[rank], one workgroup per superblock
__global__ __launch_bounds__(256) void compact_stage_kernel(const double* __restrict__ stage,
                                                            const uint32_t* __restrict__ sb_count,
                                                            uint8_t* __restrict__ img, double* __restrict__ compact) {
    __shared__ uint32_t wsum[4];
    const int64_t sb = blockIdx.x;
    uint32_t before = 0;
    for (int64_t i = threadIdx.x; i < sb; i += blockDim.x) before += sb_count[i];
    for (int off = 32; off >= 1; off >>= 1) before += __shfl_xor(before, off, kWave);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = before;
    __syncthreads();
    const uint32_t base = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (threadIdx.x == 0) {
        const int64_t part = sb / kBase32;
        uint32_t* b32 = reinterpret_cast<uint32_t*>(img + part * kImgBytes + int64_t(kWords) * 8 +
                                                    int64_t(kRank16) * 2);
        b32[sb % kBase32] = base;
    }
    const uint32_t n = sb_count[sb];
    const double* src = stage + sb * kSuper;
    for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) compact[static_cast<int64_t>(base) + k] = src[k];
}

// ---------------------------------------------------------------------------
// the sparse pool (built once, when the tables are created)
// ---------------------------------------------------------------------------

// nonzero count of every (row, 4096-event chunk); grid (n_chunks, n_rows)
__global__ __launch_bounds__(256) void sparse_count_kernel(const double* __restrict__ elts, int64_t C,
                                                           int64_t n_chunks, int64_t* __restrict__ counts) {
    __shared__ uint32_t wsum[4];
    const int64_t row = blockIdx.y, chunk = blockIdx.x;
    const double* r = elts + row * C;
    const int64_t e0 = chunk * kSuper;
    uint32_t cnt = 0;
    for (int k = 0; k < kSuper / 256; ++k) {
        const int64_t E = e0 + k * 256 + threadIdx.x;
        cnt += (E < C && __builtin_nontemporal_load(r + E) != 0.0) ? 1u : 0u;
    }
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, kWave);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) counts[row * n_chunks + chunk] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// exclusive scan of n counts in place (one workgroup), with the total at [n]
__global__ __launch_bounds__(1024) void sparse_scan_kernel(int64_t* __restrict__ v, int64_t n) {
    __shared__ int64_t sh[1024];
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < n; c0 += 1024) {
        const int64_t i = c0 + threadIdx.x;
        const int64_t x = i < n ? v[i] : 0;
        sh[threadIdx.x] = x;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int64_t add = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < n) v[i] = carry + sh[threadIdx.x] - x;
        const int64_t total = sh[1023];
        __syncthreads();
        carry += total;
    }
    if (threadIdx.x == 0) v[n] = carry;
}

// each chunk's nonzero entries, in event order, at its offset; grid (n_chunks, n_rows)
__global__ __launch_bounds__(256) void sparse_fill_kernel(const double* __restrict__ elts, int64_t C,
                                                          int64_t n_chunks, const int64_t* __restrict__ off,
                                                          uint16_t* __restrict__ ev, double* __restrict__ val) {
    __shared__ uint32_t wsum[4];
    const int64_t row = blockIdx.y, chunk = blockIdx.x;
    const double* r = elts + row * C;
    const int64_t e0 = chunk * kSuper;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t at = off[row * n_chunks + chunk];
    for (int k = 0; k < kSuper / 256; ++k) {
        const int local = k * 256 + static_cast<int>(threadIdx.x);
        const int64_t E = e0 + local;
        const double x = E < C ? r[E] : 0.0;
        const uint64_t bal = __ballot(x != 0.0);
        if (lane == 0) wsum[w] = __popcll(bal);
        __syncthreads();
        uint32_t before = 0;
        for (int i = 0; i < w; ++i) before += wsum[i];
        const uint32_t total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        if (x != 0.0) {
            const int64_t pos = at + before + __popcll(bal & lanemask_lt());
            ev[pos] = static_cast<uint16_t>(local);
            val[pos] = x;
        }
        at += total;
        __syncthreads();
    }
}

// exclusive scan of the superblock counts (one workgroup) into each part's
// base32 table
__global__ __launch_bounds__(1024) void superblock_scan_kernel(const uint32_t* __restrict__ sb_count, int64_t n_sb,
                                                               uint8_t* __restrict__ img, int64_t img_stride) {
    __shared__ uint64_t s[1024];
    sb_count += blockIdx.y * n_sb;
    img += blockIdx.y * img_stride;
    uint64_t carry = 0;
    for (int64_t c0 = 0; c0 < n_sb; c0 += 1024) {
        const int64_t i = c0 + threadIdx.x;
        const uint64_t v = i < n_sb ? sb_count[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            uint64_t add = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < n_sb) {
            const int64_t part = i / kBase32;
            const int ls = static_cast<int>(i % kBase32);
            uint32_t* b32 = reinterpret_cast<uint32_t*>(img + part * kImgBytes + int64_t(kWords) * 8 +
                                                        int64_t(kRank16) * 2);
            b32[ls] = static_cast<uint32_t>(carry + s[threadIdx.x] - v);
        }
        const uint64_t total = s[1023];
        __syncthreads();
        carry += total;
    }
}

// nonzero o(E) to compact[rank(E)], one workgroup per superblock
__global__ __launch_bounds__(256) void compact_kernel(const double* __restrict__ o, int64_t C,
                                                      const uint8_t* __restrict__ img, double* __restrict__ compact,
                                                      int64_t o_stride, int64_t img_stride) {
    __shared__ uint32_t pre[64];
    o += blockIdx.y * o_stride;
    img += blockIdx.y * img_stride;
    compact += blockIdx.y * o_stride;
    const int64_t sb = blockIdx.x;
    const int64_t e0 = sb * kSuper;
    const int64_t part = e0 >> kPartShift;
    const int ls = static_cast<int>((e0 & (kPartSize - 1)) >> kSuperShift);
    const uint64_t* bm = reinterpret_cast<const uint64_t*>(img + part * kImgBytes);
    const uint32_t* b32 = reinterpret_cast<const uint32_t*>(img + part * kImgBytes + int64_t(kWords) * 8 +
                                                            int64_t(kRank16) * 2);
    if (threadIdx.x == 0) {
        uint32_t run = b32[ls];
        for (int k = 0; k < 64; ++k) {
            pre[k] = run;
            run += __popcll(bm[ls * 64 + k]);
        }
    }
    __syncthreads();
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    for (int k = 0; k < 16; ++k) {
        const int word = w * 16 + k;
        const int64_t E = e0 + word * 64 + lane;
        const uint64_t bits = bm[ls * 64 + word];
        if ((bits >> lane) & 1ull) compact[pre[word] + __popcll(bits & lanemask_lt())] = o[E];
    }
}

// ---------------------------------------------------------------------------
// the partitioned trial pass
// ---------------------------------------------------------------------------

// LDS state of one workgroup of the partitioned pass
struct PassLds {
    uint64_t bm[kWords];
    uint16_t r16[kRank16];
    uint32_t b32[kBase32];
    double acc_hi[kTileMax];
    double acc_lo[kTileMax];
    int64_t tile;
    int32_t item;
};

// One (layer, tile): every part image in turn, every trial of the tile inside
// [t_lo, t_hi); writes YLT (and S) for those trials.  All threads of the
// workgroup call it; it starts and ends with a barrier.
template <int LPT>
__device__ __forceinline__ void pass_tile(PassLds& sh, const uint32_t* __restrict__ pids,
                                          const uint32_t* __restrict__ seg_rel,
                                          const int64_t* __restrict__ tile_start, const uint8_t* __restrict__ img,
                                          const double* __restrict__ compact, int64_t N, int P, int T, int64_t tile,
                                          int64_t t_lo, int64_t t_hi, double aggR, double aggL,
                                          double* __restrict__ ylt, double* __restrict__ S_out) {
    static_assert(LPT == 8 || LPT == 16 || LPT == 32 || LPT == 64, "lanes per trial");
    const int lig = threadIdx.x & (LPT - 1);                   // lane in its group
    const int slot = threadIdx.x / LPT;                        // group index in the workgroup
    const int n_slots = blockDim.x / LPT;
    const int64_t t0 = tile * T;
    const int Tk = static_cast<int>(N - t0 < T ? N - t0 : T);
    const int64_t sbase = tile * (static_cast<int64_t>(T) * P + 1);
    const uint32_t* tids = pids + tile_start[tile];
    for (int i = threadIdx.x; i < Tk; i += blockDim.x) {
        sh.acc_hi[i] = 0.0;
        sh.acc_lo[i] = 0.0;
    }
    for (int p = 0; p < P; ++p) {
        __syncthreads();
        {
            const u32x4* src = reinterpret_cast<const u32x4*>(img + p * kImgBytes);
            u32x4* dst_bm = reinterpret_cast<u32x4*>(sh.bm);
            for (int k = threadIdx.x; k < kWords / 2; k += blockDim.x) dst_bm[k] = src[k];
            const u32x4* src_r = src + kWords / 2;
            u32x4* dst_r = reinterpret_cast<u32x4*>(sh.r16);
            for (int k = threadIdx.x; k < kRank16 / 8; k += blockDim.x) dst_r[k] = src_r[k];
            const u32x4* src_b = src_r + kRank16 / 8;
            u32x4* dst_b = reinterpret_cast<u32x4*>(sh.b32);
            for (int k = threadIdx.x; k < kBase32 / 4; k += blockDim.x) dst_b[k] = src_b[k];
        }
        __syncthreads();
        const uint32_t pbase = static_cast<uint32_t>(static_cast<int64_t>(p) << kPartShift);
        // A group walks its trials' segments of this part in batches of
        // LPT*4*kU IDs; the loads of the next batch are issued before the
        // current batch is looked up, so HBM latency overlaps the LDS tests,
        // the gathers and the sums.  Trials outside [t_lo, t_hi) have empty
        // segments.
        constexpr int kU = 4;
        constexpr uint32_t kBatch = LPT * 4 * kU;
        auto seg = [&](int i, uint32_t& sb, uint32_t& se) {
            const int64_t t = t0 + i;
            sb = seg_rel[sbase + static_cast<int64_t>(p) * Tk + i];
            se = (t < t_lo || t >= t_hi) ? sb : seg_rel[sbase + static_cast<int64_t>(p) * Tk + i + 1];
        };
        auto load_batch = [&](uint32_t c, uint32_t e, u32x4* v) {
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const uint32_t cu = c + lig * 4 + u * LPT * 4;
                v[u] = cu < e ? __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(tids + cu))
                              : u32x4{kSentinel, kSentinel, kSentinel, kSentinel};
            }
        };
        int i = slot;
        uint32_t cs = 0, ce = 0, c = 0;
        u32x4 cur[kU], nxt[kU];
        if (i < Tk) {
            seg(i, cs, ce);
            c = cs;
            load_batch(c, ce, cur);
        }
        double hi = 0.0, lo = 0.0;
        while (i < Tk) {
            // coordinates of the next batch: the rest of this segment, or the
            // group's next trial
            int ni = i;
            uint32_t ns = cs, ne = ce, nc = c + kBatch;
            if (nc >= ce) {
                ni = i + n_slots;
                if (ni < Tk) {
                    seg(ni, ns, ne);
                    nc = ns;
                }
            }
            if (ni < Tk) load_batch(nc, ne, nxt);
            uint32_t r[kU * 4];
#pragma unroll
            for (int k = 0; k < kU * 4; ++k) {
                const uint32_t el = cur[k >> 2][k & 3] - pbase;   // sentinel and foreign IDs fail the test
                r[k] = 0xFFFFFFFFu;
                if (el < static_cast<uint32_t>(kPartSize)) {
                    const uint64_t word = sh.bm[el >> 6];
                    if ((word >> (el & 63)) & 1ull) {
                        uint32_t rk = sh.b32[el >> kSuperShift] + sh.r16[el >> 7];
                        if ((el >> 6) & 1) rk += __popcll(sh.bm[(el >> 6) - 1]);
                        r[k] = rk + __popcll(word & ((1ull << (el & 63)) - 1ull));
                    }
                }
            }
            double val[kU * 4];
#pragma unroll
            for (int k = 0; k < kU * 4; ++k) val[k] = compact[r[k] == 0xFFFFFFFFu ? 0u : r[k]];
#pragma unroll
            for (int k = 0; k < kU * 4; ++k) dd_add(hi, lo, r[k] == 0xFFFFFFFFu ? 0.0 : val[k]);
            if (ni != i) {
                // the trial's segment is done: group total into its accumulator
                group_reduce_dd(hi, lo, LPT);
                if (lig == 0) {
                    double h = sh.acc_hi[i], l = sh.acc_lo[i];
                    dd_merge(h, l, hi, lo);
                    sh.acc_hi[i] = h;
                    sh.acc_lo[i] = l;
                }
                hi = 0.0;
                lo = 0.0;
            }
            i = ni;
            cs = ns;
            ce = ne;
            c = nc;
#pragma unroll
            for (int u = 0; u < kU; ++u) cur[u] = nxt[u];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < Tk; i += blockDim.x) {
        const int64_t t = t0 + i;
        if (t < t_lo || t >= t_hi) continue;
        const double S = sh.acc_hi[i] + sh.acc_lo[i];
        ylt[t - t_lo] = apply_terms(S, aggR, aggL);
        if (S_out) S_out[t - t_lo] = S;
    }
    __syncthreads();
}

template <int LPT>
__global__ __launch_bounds__(512) void part_pass_kernel(PartPassArgs a) {
    __shared__ __attribute__((aligned(16))) PassLds sh;
    for (;;) {
        if (threadIdx.x == 0) sh.tile = a.first_tile + atomicAdd(a.tile_counter, 1u);
        __syncthreads();
        const int64_t tile = sh.tile;
        if (tile >= a.last_tile) break;
        pass_tile<LPT>(sh, a.pids, a.seg_rel, a.tile_start, a.img, a.compact, a.N, a.P, a.T, tile, a.t_lo,
                       a.t_hi, a.aggR, a.aggL, a.ylt, a.S);
    }
}

// The persistent multi-layer pass: one grid drains a work list of
// (layer, tile) items, ordered by decreasing cost, through an atomic counter.
template <int LPT>
__global__ __launch_bounds__(512) void batched_pass_kernel(BatchedPassArgs a) {
    __shared__ __attribute__((aligned(16))) PassLds sh;
    for (;;) {
        if (threadIdx.x == 0) sh.item = static_cast<int32_t>(atomicAdd(a.item_counter, 1u));
        __syncthreads();
        const int32_t it = sh.item;
        if (it >= a.n_items) break;
        const int2 w = a.items[it];
        const BatchLayerDesc d = a.layers[w.x];
        pass_tile<LPT>(sh, a.pids, a.seg_rel, a.tile_start, a.img + w.x * a.img_stride, a.compact + w.x * a.C,
                       a.N, a.P, a.T, w.y, d.t_lo, d.t_hi, d.aggR, d.aggL, a.ylt + d.out_off, nullptr);
    }
}

// per-layer fold for a batch: o[l][E], ELT terms from device tables
__global__ __launch_bounds__(256) void batched_fold_kernel(const double* __restrict__ elts, int64_t C,
                                                           const BatchFoldDesc* __restrict__ fd,
                                                           const int32_t* __restrict__ idx,
                                                           const double* __restrict__ R,
                                                           const double* __restrict__ Lim, double* __restrict__ o) {
    const int l = blockIdx.y;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= C) return;
    const BatchFoldDesc d = fd[l];
    double y = 0.0;
    for (int j = 0; j < d.J; ++j) {
        const int k = d.off + j;
        y = y + apply_terms(elts[static_cast<int64_t>(idx[k]) * C + e], R[k], Lim[k]);
    }
    o[static_cast<int64_t>(l) * C + e] = apply_terms(y, d.occR, d.occL);
}

// Backward histogram over the partitioned layout: for every trial inside the
// aggregate band, every occurrence whose event has a movable occurrence loss
// (bit set in the part bitmap) adds 1 to W_mean[E] and the trial's TVaR weight
// to W_tvar[E].  Integer atomics: the histogram does not depend on order.
__global__ __launch_bounds__(512) void part_adjoint_kernel(PartAdjArgs a) {
    __shared__ __attribute__((aligned(16))) uint64_t bm[kWords];
    __shared__ int64_t s_tile;
    const int lane = threadIdx.x & 63;
    const int lig = lane & 15;
    const int slot = (threadIdx.x >> 6) * 4 + (lane >> 4);
    const int P = a.P;
    const TailStats ts = *a.tail;
    for (;;) {
        if (threadIdx.x == 0) s_tile = a.first_tile + atomicAdd(a.tile_counter, 1u);
        __syncthreads();
        const int64_t tile = s_tile;
        if (tile >= a.last_tile) break;
        const int64_t t0 = tile * a.T;
        const int Tk = static_cast<int>(a.N - t0 < a.T ? a.N - t0 : a.T);
        const int64_t sbase = tile * (static_cast<int64_t>(a.T) * P + 1);
        const uint32_t* tids = a.pids + a.tile_start[tile];
        for (int p = 0; p < P; ++p) {
            __syncthreads();
            {
                const u32x4* src = reinterpret_cast<const u32x4*>(a.img + p * kImgBytes);
                u32x4* dst = reinterpret_cast<u32x4*>(bm);
                for (int k = threadIdx.x; k < kWords / 2; k += blockDim.x) dst[k] = src[k];
            }
            __syncthreads();
            const uint32_t pbase = static_cast<uint32_t>(static_cast<int64_t>(p) << kPartShift);
            for (int i = slot; i < Tk; i += 32) {
                const int64_t t = t0 + i;
                if (t < a.t_lo || t >= a.t_hi) continue;
                const int64_t k = t - a.t_lo;
                const double ta = a.S[k] - a.aggR;
                if (!((ta > 0.0) && (ta < a.aggL))) continue;
                const uint64_t key = __double_as_longlong(a.ylt[k] + 0.0);
                const unsigned long long wt =
                    key > ts.v_bits ? ts.c_eq : (key == ts.v_bits ? ts.m - ts.c_gt : 0);
                const uint32_t s = a.seg_rel[sbase + static_cast<int64_t>(p) * Tk + i];
                const uint32_t e = a.seg_rel[sbase + static_cast<int64_t>(p) * Tk + i + 1];
                constexpr int kU = 4;
                for (uint32_t c = s + lig * 4; c < e; c += 64 * kU) {
                    u32x4 v[kU];
#pragma unroll
                    for (int u = 0; u < kU; ++u) {
                        const uint32_t cu = c + u * 64;
                        v[u] = cu < e ? __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(tids + cu))
                                      : u32x4{kSentinel, kSentinel, kSentinel, kSentinel};
                    }
#pragma unroll
                    for (int k = 0; k < kU * 4; ++k) {
                        const uint32_t id = v[k >> 2][k & 3];
                        const uint32_t el = id - pbase;
                        if (el < static_cast<uint32_t>(kPartSize) && ((bm[el >> 6] >> (el & 63)) & 1ull)) {
                            atomicAdd(reinterpret_cast<unsigned long long*>(&a.w_mean[id]), 1ull);
                            if (wt) atomicAdd(reinterpret_cast<unsigned long long*>(&a.w_tvar[id]), wt);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Backward histogram, XCD-affine, for the same result as part_adjoint_kernel.
// Workgroups on XCD x serve the parts p = x (mod 8) as in the forward pass,
// each over a fixed share of the tiles, so a part's probe words (bitmap bits
// and part-relative ranks, built from the part image and its superblock
// counts) are loaded into LDS once.  An occurrence of a movable event in a
// trial inside the aggregate band counts 1 for W_mean: in an LDS counter
// when the event is among the part's first kCounts nonzero events (by rank),
// else with a global atomic; the LDS counters are added to W_mean once per
// part.  TVaR weights (tail trials only) use global atomics.  Each group of
// 16 lanes takes four trials of a tile at once, so their segments' loads are
// in flight together.  All counts are integers, so the order of the additions
// does not matter.  The LDS counters
// are 32-bit: the launcher uses this kernel only for layouts of fewer than
// 2^32 IDs, which bounds every count.
__global__ __launch_bounds__(1024) void xcd_adjoint_kernel(PartAdjArgs a, int n_xcd) {
    constexpr uint32_t kProbeWords = static_cast<uint32_t>(kPartSize >> 5);
    constexpr uint32_t kCounts = 24000;
    __shared__ uint64_t pw[kProbeWords];
    __shared__ uint32_t cnt[kCounts];
    __shared__ uint32_t sbb[kBase32];               // part-relative rank of each superblock's first event
    const int lane = threadIdx.x & 63;
    const int lig = lane & 15;
    const int slot = (threadIdx.x >> 6) * 4 + (lane >> 4);     // 64 groups of 16 lanes, one trial each
    const int n_slots = static_cast<int>(blockDim.x >> 4);
    const int P = a.P;
    const TailStats ts = *a.tail;
    const int x = static_cast<int>(blockIdx.x % n_xcd);
    const int r = static_cast<int>(blockIdx.x / n_xcd);
    const int nr = static_cast<int>(gridDim.x / n_xcd);
    int p0, pstep, srank, nserv;
    if (P >= n_xcd) {
        p0 = x;
        pstep = n_xcd;
        srank = r;
        nserv = nr;
    } else {
        p0 = x % P;
        pstep = P;
        srank = (x / P) * nr + r;
        nserv = ((n_xcd - 1 - p0) / P + 1) * nr;
    }
    const int64_t n_tiles = a.last_tile - a.first_tile;
    for (int p = p0; p < P; p += pstep) {
        const uint8_t* gimg = a.img + static_cast<int64_t>(p) * kImgBytes;
        const uint32_t* gbm = reinterpret_cast<const uint32_t*>(gimg);
        const uint16_t* gr16 = reinterpret_cast<const uint16_t*>(gimg + int64_t(kWords) * 8);
        __syncthreads();                            // the previous part's counters are flushed
        if (threadIdx.x == 0) {
            uint32_t run = 0;
            for (int k = 0; k < kBase32; ++k) {
                sbb[k] = run;
                run += a.sb_count[static_cast<int64_t>(p) * kBase32 + k];
            }
        }
        for (uint32_t k = threadIdx.x; k < kCounts; k += blockDim.x) cnt[k] = 0;
        __syncthreads();
        for (uint32_t j = threadIdx.x; j < kProbeWords; j += blockDim.x) {
            uint32_t rank = sbb[j >> 7] + gr16[j >> 2];
            for (uint32_t k = j & ~3u; k < j; ++k) rank += __builtin_popcount(gbm[k]);
            pw[j] = (static_cast<uint64_t>(rank) << 32) | gbm[j];
        }
        __syncthreads();
        const uint32_t pbase = static_cast<uint32_t>(static_cast<int64_t>(p) << kPartShift);
        for (int64_t m = srank; m < n_tiles; m += nserv) {
            const int64_t tile = a.first_tile + m;
            const int64_t t0 = tile * a.T;
            const int Tk = static_cast<int>(a.N - t0 < a.T ? a.N - t0 : a.T);
            const int64_t sbase = tile * (static_cast<int64_t>(a.T) * P + 1);
            const uint32_t* tids = a.pids + a.tile_start[tile];
            // kTr trials per group of 16 lanes, whose segments' loads are in flight together
            constexpr int kTr = 4;
            for (int i0 = slot; i0 < Tk; i0 += kTr * n_slots) {
                uint32_t sb2[kTr], len2[kTr];
                unsigned long long wt2[kTr];
#pragma unroll
                for (int h = 0; h < kTr; ++h) {
                    const int i = i0 + h * n_slots;
                    sb2[h] = 0;
                    len2[h] = 0;
                    wt2[h] = 0;
                    const int64_t t = t0 + i;
                    if (i >= Tk || t < a.t_lo || t >= a.t_hi) continue;
                    const int64_t k = t - a.t_lo;
                    const double ta = a.S[k] - a.aggR;
                    if (!((ta > 0.0) && (ta < a.aggL))) continue;        // outside the aggregate band
                    const uint64_t key = __double_as_longlong(a.ylt[k] + 0.0);
                    wt2[h] = key > ts.v_bits ? ts.c_eq : (key == ts.v_bits ? ts.m - ts.c_gt : 0);
                    sb2[h] = a.seg_rel[sbase + static_cast<int64_t>(p) * Tk + i];
                    len2[h] = a.seg_rel[sbase + static_cast<int64_t>(p) * Tk + i + 1] - sb2[h];
                }
                constexpr int kU = 4;
                uint32_t lmax = 0;
#pragma unroll
                for (int h = 0; h < kTr; ++h) lmax = len2[h] > lmax ? len2[h] : lmax;
                for (uint32_t off = lig * 4; off < lmax; off += 64 * kU) {
                    u32x4 v[kTr][kU];
#pragma unroll
                    for (int h = 0; h < kTr; ++h)
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const uint32_t o = off + u * 64;
                            v[h][u] = o < len2[h]
                                          ? __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(tids + sb2[h] + o))
                                          : u32x4{kSentinel, kSentinel, kSentinel, kSentinel};
                        }
#pragma unroll
                    for (int h = 0; h < kTr; ++h)
#pragma unroll
                        for (int q = 0; q < kU * 4; ++q) {
                            const uint32_t id = v[h][q >> 2][q & 3];
                            const uint32_t el = id - pbase;
                            if (el >= static_cast<uint32_t>(kPartSize)) continue;     // padding
                            const uint64_t w = pw[el >> 5];
                            const uint32_t bi = el & 31u;
                            if (!((w >> bi) & 1ull)) continue;
                            const uint32_t rank = static_cast<uint32_t>(w >> 32) +
                                                  __builtin_popcount(static_cast<uint32_t>(w) & ((1u << bi) - 1u));
                            if (rank < kCounts)
                                atomicAdd(&cnt[rank], 1u);
                            else
                                atomicAdd(reinterpret_cast<unsigned long long*>(&a.w_mean[id]), 1ull);
                            if (wt2[h]) atomicAdd(reinterpret_cast<unsigned long long*>(&a.w_tvar[id]), wt2[h]);
                        }
                }
            }
        }
        __syncthreads();
        // the LDS counters to W_mean: the events of each probe word, in rank order
        for (uint32_t j = threadIdx.x; j < kProbeWords; j += blockDim.x) {
            const uint64_t w = pw[j];
            uint32_t bits = static_cast<uint32_t>(w);
            uint32_t rank = static_cast<uint32_t>(w >> 32);
            while (bits && rank < kCounts) {
                const uint32_t b = static_cast<uint32_t>(__builtin_ctz(bits));
                const uint32_t c = cnt[rank];
                if (c) atomicAdd(reinterpret_cast<unsigned long long*>(&a.w_mean[pbase + j * 32 + b]),
                                 static_cast<unsigned long long>(c));
                bits &= bits - 1u;
                ++rank;
            }
        }
    }
}

// XCD-affine pass.  Workgroups are dispatched to the 8 XCDs round-robin, so
// workgroup b runs on XCD b % 8; each XCD serves its own catalogue parts
// (part p on XCD p % 8).  A part's dense occurrence losses are 2 MB, so they
// stay in that XCD's 4 MB L2 and a hit gathers o[E] directly, with no rank
// arithmetic; the part's 32 KB bitmap is loaded into LDS once per part.  Each
// (part, trial) double-double partial goes to HBM; xcd_combine_kernel adds
// the parts of a trial in part order.
// Inclusive prefix sum over the 64 lanes of a wave with DPP lane moves: four
// shifts build each 16-lane row's scan, two row broadcasts carry row totals.
__device__ __forceinline__ uint32_t wave_scan_u32(uint32_t x) {
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x111, 0xF, 0xF, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x112, 0xF, 0xF, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x114, 0xF, 0xF, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x118, 0xF, 0xF, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x142, 0xA, 0xF, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x143, 0xC, 0xF, false));
    return x;
}

// the value held by the partner lane (lane ^ 1)
__device__ __forceinline__ double swap_pair_f64(double v) {
    const uint64_t b = __double_as_longlong(v);
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(static_cast<uint32_t>(b)), 0xB1,
                                                                        0xF, 0xF, false));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(static_cast<uint32_t>(b >> 32)),
                                                                        0xB1, 0xF, 0xF, false));
    return __longlong_as_double(static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo));
}

// XCD-affine trial pass.  Workgroups on XCD x serve the catalogue parts
// p = x (mod 8), whose 2 MB of occurrence losses stay in that XCD's L2.  Each
// wave owns 32 consecutive trials of a tile and streams their IDs of part p
// as one contiguous range, 1024 IDs per batch: every ID is tested against the
// part's bitmap in LDS and the hits are appended, in position order, to the
// wave's LDS queue.  The queue is drained at the end of the tile (or when it
// may overflow): two lanes per trial gather the losses of that trial's hits
// and sum them in double-double, in queue order, so the result does not
// depend on timing.  Tiles are assigned to workgroups statically, so the
// next tile's boundaries are read a tile ahead and its first batch is loaded
// while the current tile's last one is tested.
__global__ __launch_bounds__(1024) void xcd_pass_kernel(XcdPassArgs a) {
    constexpr int kU = 2;                           // 16-byte loads per lane per batch
    constexpr int kTrialsPW = kTileMax / 8;         // 32 trials per wave
    constexpr uint32_t kBatch = 64 * 4 * kU;        // IDs per batch
    constexpr int kQ = 512;                         // queue entries per wave (one batch)
    constexpr int kInf = 0x3FFFFFFF;
    static_assert(kQ >= static_cast<int>(kBatch), "a batch must fit the queue");
    // LDS, one block: the part's probe words (one per 32 events: the bitmap
    // bits in the low half, the part-relative rank of the word's first event
    // among the nonzero ones in the high half) -- first, so a probe word's
    // byte offset is its LDS address -- then the hit queues, then as many of
    // the part's first nonzero losses as fit
    constexpr uint32_t kProbeWords = static_cast<uint32_t>(kPartSize >> 5);
    constexpr uint32_t kProbeMask = (kProbeWords - 1) * 8;              // byte offset bits of a probe word
    constexpr uint32_t kQueueOff = kProbeWords * 8;                     // 16 per-wave hit queues (event IDs)
    constexpr uint32_t kCacheOff = kQueueOff + 16 * kQ * 4;             // the loss cache (8-byte aligned)
    constexpr int kCache = static_cast<int>((160 * 1024 - kCacheOff) / 8);
    static_assert(kCacheOff % 16 == 0 && kCache > 0, "LDS layout");
    __shared__ __attribute__((aligned(16))) uint8_t lds[kCacheOff + kCache * 8];
    uint64_t* pwords = reinterpret_cast<uint64_t*>(lds);
    double* cache = reinterpret_cast<double*>(lds + kCacheOff);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    uint32_t* q = reinterpret_cast<uint32_t*>(lds + kQueueOff) + wv * kQ;
    // parts served by this workgroup (its XCD's), and its rank among the servers
    // of each; the two halves of the workgroup (8 waves each) serve separately
    const int n_xcd = a.n_xcd;
    const int x = static_cast<int>(blockIdx.x % n_xcd);
    const int r = static_cast<int>(blockIdx.x / n_xcd);
    const int nr = static_cast<int>(gridDim.x / n_xcd);
    const int P = a.P;
    int p0, pstep, srank, nserv;
    if (P >= n_xcd) {
        p0 = x;
        pstep = n_xcd;
        srank = r;
        nserv = nr;
    } else {
        p0 = x % P;
        pstep = P;
        srank = (x / P) * nr + r;
        nserv = ((n_xcd - 1 - p0) / P + 1) * nr;
    }
    srank = 2 * srank + (wv >> 3);
    nserv = 2 * nserv;
    const int64_t n_tiles = a.last_tile - a.first_tile;
    const int64_t count = a.t_hi - a.t_lo;
    const int j0w = (wv & 7) * kTrialsPW;           // the wave's first trial in a tile
    const int pt = lane >> 1;                       // the trial this lane sums (with its partner)
    const int half = lane & 1;

    for (int p = p0; p < P; p += pstep) {
        // the part image (bitmap, 128-event ranks within superblocks, global
        // superblock ranks) becomes the probe words
        const uint8_t* gimg = a.img + static_cast<int64_t>(p) * kImgBytes;
        const uint32_t* gbm = reinterpret_cast<const uint32_t*>(gimg);
        const uint16_t* gr16 = reinterpret_cast<const uint16_t*>(gimg + int64_t(kWords) * 8);
        const uint32_t* gb32 = reinterpret_cast<const uint32_t*>(gimg + int64_t(kWords) * 8 + int64_t(kRank16) * 2);
        const uint32_t rank0 = gb32[0];             // global rank of the part's first nonzero loss
        __syncthreads();
        for (uint32_t j = threadIdx.x; j < kProbeWords; j += blockDim.x) {
            uint32_t rank = gb32[j >> 7] - rank0 + gr16[j >> 2];
            for (uint32_t k = j & ~3u; k < j; ++k) rank += __builtin_popcount(gbm[k]);
            pwords[j] = (static_cast<uint64_t>(rank) << 32) | gbm[j];
        }
        __syncthreads();
        // the part's first nonzero losses, in rank order
        for (int k = threadIdx.x; k < kCache; k += blockDim.x) {
            const int64_t g = static_cast<int64_t>(rank0) + k;
            cache[k] = g < a.C ? a.compact[g] : 0.0;
        }
        __syncthreads();
        if (srank >= n_tiles) continue;

        // this server's m-th tile, clamped to a real tile past the end (never used there)
        auto tile_of = [&](int64_t m) -> int64_t {
            const int64_t tile = a.first_tile + srank + m * nserv;
            return tile < a.last_tile ? tile : a.last_tile - 1;
        };
        auto trials_in = [&](int64_t tile) -> int {
            const int64_t t0 = tile * a.T;
            return static_cast<int>(a.N - t0 < a.T ? a.N - t0 : a.T);
        };
        // the wave's 33 segment boundaries in a tile, lane i holding boundary i
        // (lanes past 32 repeat the last), clamped to the tile's trial count
        auto load_bounds = [&](int64_t tile) -> uint32_t {
            const int Tk = trials_in(tile);
            const int64_t sb = tile * (static_cast<int64_t>(a.T) * P + 1) + static_cast<int64_t>(p) * Tk;
            const int i = j0w + (lane < kTrialsPW ? lane : kTrialsPW);
            return a.seg_rel[sb + (i < Tk ? i : Tk)];
        };
        // the wave's trials [jlo, jhi) of a tile (relative to j0w), clipped to
        // the tile and to the layer's trials
        auto clip = [&](int64_t tile, int& jlo, int& jhi) {
            const int64_t t0 = tile * a.T + j0w;
            const int Tk = trials_in(tile) - j0w;
            jlo = 0;
            jhi = kTrialsPW < Tk ? kTrialsPW : (Tk > 0 ? Tk : 0);
            if (t0 + jlo < a.t_lo) jlo = static_cast<int>(a.t_lo - t0 < jhi ? a.t_lo - t0 : jhi);
            if (t0 + jhi > a.t_hi) jhi = static_cast<int>(a.t_hi - t0 > jlo ? a.t_hi - t0 : jlo);
            if (jhi < jlo) jhi = jlo;
        };

        // current tile
        int64_t m = 0;
        int64_t tile = tile_of(0);
        uint32_t B = load_bounds(tile);
        int jlo, jhi;
        uint32_t rs, re;
        const uint32_t* tids;
        // next tile: its range and ID base (its first batch is loaded during
        // this tile's last); boundaries of the next two tiles are read ahead
        uint32_t B1 = load_bounds(tile_of(1));
        uint32_t B2 = load_bounds(tile_of(2));
        uint32_t n_rs, n_re;
        const uint32_t* n_tids;
        bool has_next = srank + nserv < n_tiles;
        int qs;                                     // lane i: queue index of trial i's first hit
        int qn = 0;                                 // entries in the queue
        double acc_hi = 0.0, acc_lo = 0.0;

        auto enter = [&]() {                        // make `tile` (boundaries B) current
            clip(tile, jlo, jhi);
            rs = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(B), jlo));
            re = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(B), jhi));
            tids = a.pids + a.tile_start[tile];
            qs = B <= rs ? 0 : kInf;
        };
        auto aim = [&](int64_t ntile) {             // the range of `ntile` (boundaries B1)
            int nlo, nhi;
            clip(ntile, nlo, nhi);
            n_rs = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(B1), nlo));
            n_re = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(B1), nhi));
            n_tids = a.pids + a.tile_start[ntile];
        };
        enter();
        aim(tile_of(1));
        // batches start on 128-byte lines (tiles are aligned); positions before
        // rs are masked off
        uint32_t c = rs & ~uint32_t(kTileAlign - 1);

        // one batch of 16-byte ID chunks; chunks at or past `end` read the
        // padding instead (cached), so no HBM line past the range is fetched
        auto load_batch = [&](const uint32_t* ids, uint32_t cb, uint32_t end, u32x4* v) {
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const uint32_t cu = cb + u * 256 + lane * 4;
                const uint32_t* src = cu < end ? ids + cu : a.pad;
                v[u] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(src));
            }
        };
        // the batch after the one at c: the rest of this tile, else the next tile's first
        auto load_next = [&](u32x4* v) {
            if (c + kBatch < re)
                load_batch(tids, c + kBatch, re, v);
            else
                load_batch(n_tids, n_rs & ~uint32_t(kTileAlign - 1), has_next ? n_re : 0u, v);
        };
        // gather and sum the queued hits: lanes 2t and 2t+1 take trial t's
        // entries alternately, four gathers in flight per lane
        auto drain = [&]() {
            int lo = __shfl(qs, pt), hi = __shfl(qs, pt + 1);
            lo = lo < 0 ? 0 : (lo > qn ? qn : lo);
            hi = hi < 0 ? 0 : (hi > qn ? qn : hi);
            for (int j = lo + half; j < hi; j += 8) {
                double v[4];
#pragma unroll
                for (int r2 = 0; r2 < 4; ++r2) {
                    const int jj = j + 2 * r2;
                    v[r2] = 0.0;
                    if (jj < hi) {
                        // rank of the event among the part's nonzero ones: its probe
                        // word's, plus the set bits below it in the word.  Parts are
                        // aligned, so the low bits of an ID are its part-relative
                        // index; a queued padding ID reads as the part's last event.
                        const uint32_t id = q[jj];
                        const uint32_t e = id & static_cast<uint32_t>(kPartSize - 1);
                        const uint64_t pwd = *reinterpret_cast<const uint64_t*>(lds + (e >> 5) * 8u);
                        const uint32_t below = (1u << (e & 31u)) - 1u;
                        const uint32_t lr = static_cast<uint32_t>(pwd >> 32) +
                                            __builtin_popcount(static_cast<uint32_t>(pwd) & below);
                        // the LDS copy, read at a clamped rank, else the value from L2
                        // (two loads of one address space each, no pointer select)
                        v[r2] = cache[min(lr, static_cast<uint32_t>(kCache - 1))];
                        if (lr >= static_cast<uint32_t>(kCache)) v[r2] = a.compact[rank0 + lr];
                        if (id == kSentinel) v[r2] = 0.0;   // segment padding adds nothing
                    }
                }
                // entries past the trial's last are 0.0, whose sum is exact
#pragma unroll
                for (int r2 = 0; r2 < 4; ++r2) dd_add(acc_hi, acc_lo, v[r2]);
            }
            qs = qs == kInf ? kInf : qs - qn;
            qn = 0;
            __builtin_amdgcn_wave_barrier();
        };
        // test a batch against the bitmap and append its hits to the queue in
        // position order (chunk u, lane, word); note where each trial's hits start
        auto process = [&](const u32x4* ids) {
            // every ID in [rs, re) belongs to part p, and parts are aligned to
            // their size, so an ID's bits 5..17 are its probe word and its low 5
            // bits the bit in it.  The only other IDs are the segment padding,
            // which reads the part's last event: if that event is nonzero the
            // padding is queued like a hit, and the drain gives it 0.0.
            uint32_t hit[kU][4];                    // word w of chunk u is a hit (0 or 1)
            uint32_t cnt[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                // a chunk lies wholly inside or outside [rs, re): both are multiples of 4
                const uint32_t ok = c + u * 256 + lane * 4 - rs < re - rs ? 1u : 0u;
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const uint32_t id = ids[u][w];
                    const uint32_t wa = (id >> 2) & kProbeMask;   // byte address of its probe word
                    const uint32_t word = *reinterpret_cast<const uint32_t*>(lds + wa);
                    hit[u][w] = __builtin_amdgcn_ubfe(word, id, 1u) & ok;
                }
                cnt[u] = hit[u][0] + hit[u][1] + hit[u][2] + hit[u][3];
            }
            // per-chunk hit counts, prefix-summed over the wave two chunks at a time
            // (16-bit halves: at most 4 x 64 hits per chunk)
            uint32_t ex[kU], tot[kU];
#pragma unroll
            for (int u = 0; u < kU; u += 2) {
                const uint32_t ha = cnt[u];
                const uint32_t hb = u + 1 < kU ? cnt[u + 1] : 0u;
                const uint32_t sc = wave_scan_u32(ha | (hb << 16));
                const uint32_t tt = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(sc), 63));
                ex[u] = (sc & 0xFFFFu) - ha;
                tot[u] = tt & 0xFFFFu;
                if (u + 1 < kU) {
                    ex[u + 1] = (sc >> 16) - hb;
                    tot[u + 1] = tt >> 16;
                }
            }
            int total = 0;
#pragma unroll
            for (int u = 0; u < kU; ++u) total += static_cast<int>(tot[u]);
            if (qn + total > kQ) drain();            // exact: the batch always fits an empty queue
            int pre[kU];
            {
                int base = qn;
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    pre[u] = base + static_cast<int>(ex[u]);
                    base += static_cast<int>(tot[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                int at = pre[u];
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    if (hit[u][w]) q[at] = ids[u][w];
                    at += static_cast<int>(hit[u][w]);
                }
            }
            // trial boundaries inside this batch: the first hit at or after the
            // boundary's chunk is where that trial's hits start
            const uint32_t k = (B - c) >> 2;        // chunk of this lane's boundary (if in the batch)
            const int src = static_cast<int>(k & 63u);
            int vq = 0;
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int v = __shfl(pre[u], src);
                vq = (k >> 6) == static_cast<uint32_t>(u) ? v : vq;
            }
            if (B > rs && B < re && B >= c && B - c < kBatch) qs = vq;
            qn += total;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };
        // after a batch: advance; at the end of the wave's range drain the queue,
        // write the trial sums and move to the next tile (its first batch is in
        // flight).  Returns false when the server's tiles are done.
        auto step = [&]() -> bool {
            c += kBatch;
            if (c < re) return true;
            drain();
            dd_merge(acc_hi, acc_lo, swap_pair_f64(acc_hi), swap_pair_f64(acc_lo));
            if (half == 0 && pt >= jlo && pt < jhi) {
                const int64_t t = tile * a.T + j0w + pt;
                a.part_hi[static_cast<int64_t>(p) * count + (t - a.t_lo)] = acc_hi;
                a.part_lo[static_cast<int64_t>(p) * count + (t - a.t_lo)] = acc_lo;
            }
            acc_hi = 0.0;
            acc_lo = 0.0;
            if (!has_next) return false;
            ++m;
            tile = tile_of(m);
            B = B1;
            enter();
            c = rs & ~uint32_t(kTileAlign - 1);
            has_next = srank + (m + 1) * nserv < n_tiles;
            B1 = B2;
            aim(tile_of(m + 1));
            B2 = load_bounds(tile_of(m + 2));
            return true;
        };

        // two register buffers in turn, so the loads of the next batch stay in
        // flight while this one is tested, with no copy that waits for them
        u32x4 bufA[kU], bufB[kU];
        load_batch(tids, c, re, bufA);
        for (;;) {
            load_next(bufB);
            process(bufA);
            if (!step()) break;
            load_next(bufA);
            process(bufB);
            if (!step()) break;
        }
    }
}

__global__ __launch_bounds__(256) void xcd_combine_kernel(const double* __restrict__ part_hi,
                                                          const double* __restrict__ part_lo, int P, int64_t count,
                                                          double aggR, double aggL, const LayerArgs* __restrict__ L_dev,
                                                          double* __restrict__ ylt, double* __restrict__ S_out) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= count) return;
    if (L_dev) {                                    // terms from device memory (graph replays)
        aggR = L_dev->aggR;
        aggL = L_dev->aggL;
    }
    double hi = 0.0, lo = 0.0;
    for (int p = 0; p < P; ++p) dd_merge(hi, lo, part_hi[p * count + k], part_lo[p * count + k]);
    const double S = hi + lo;
    ylt[k] = apply_terms(S, aggR, aggL);
    if (S_out) S_out[k] = S;
}


hipError_t launch_part_pass_lpt(int lpt, int grid, const PartPassArgs& a, hipStream_t s) {
    switch (lpt) {
        case 8: hipLaunchKernelGGL(part_pass_kernel<8>, dim3(grid), dim3(512), 0, s, a); break;
        case 32: hipLaunchKernelGGL(part_pass_kernel<32>, dim3(grid), dim3(512), 0, s, a); break;
        case 64: hipLaunchKernelGGL(part_pass_kernel<64>, dim3(grid), dim3(512), 0, s, a); break;
        default: hipLaunchKernelGGL(part_pass_kernel<16>, dim3(grid), dim3(512), 0, s, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_batched_pass_lpt(int lpt, int grid, const BatchedPassArgs& a, hipStream_t s) {
    switch (lpt) {
        case 8: hipLaunchKernelGGL(batched_pass_kernel<8>, dim3(grid), dim3(512), 0, s, a); break;
        case 32: hipLaunchKernelGGL(batched_pass_kernel<32>, dim3(grid), dim3(512), 0, s, a); break;
        case 64: hipLaunchKernelGGL(batched_pass_kernel<64>, dim3(grid), dim3(512), 0, s, a); break;
        default: hipLaunchKernelGGL(batched_pass_kernel<16>, dim3(grid), dim3(512), 0, s, a); break;
    }
    return hipGetLastError();
}

}  // namespace

int64_t part_image_bytes(int P) { return static_cast<int64_t>(P) * kImgBytes; }

hipError_t build_sparse_pool(const double* elts, int32_t n_rows, int64_t C, hipStream_t s, SparsePool* out) {
    *out = SparsePool{};
    if (n_rows > 65535) return hipErrorInvalidValue;            // rows are the grid's second dimension
    const int64_t n_chunks = (C + kSuper - 1) / kSuper;
    const int64_t n = static_cast<int64_t>(n_rows) * n_chunks;
    out->n_chunks = n_chunks;
    hipError_t e;
    if ((e = hipMalloc(&out->chunk_off, sizeof(int64_t) * (n + 1))) != hipSuccess) return e;
    out->bytes = static_cast<int64_t>(sizeof(int64_t)) * (n + 1);
    if (n == 0) return hipMemsetAsync(out->chunk_off, 0, sizeof(int64_t), s);
    const dim3 grid(static_cast<uint32_t>(n_chunks), static_cast<uint32_t>(n_rows));
    hipLaunchKernelGGL(sparse_count_kernel, grid, dim3(256), 0, s, elts, C, n_chunks, out->chunk_off);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(sparse_scan_kernel, dim3(1), dim3(1024), 0, s, out->chunk_off, n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int64_t nnz = 0;
    if ((e = hipMemcpyAsync(&nnz, out->chunk_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return e;
    out->nnz = nnz;
    const int64_t cap = nnz > 0 ? nnz : 1;
    if ((e = hipMalloc(&out->ev, sizeof(uint16_t) * cap)) != hipSuccess) return e;
    if ((e = hipMalloc(&out->val, sizeof(double) * cap)) != hipSuccess) return e;
    out->bytes += static_cast<int64_t>(sizeof(uint16_t) + sizeof(double)) * cap;
    hipLaunchKernelGGL(sparse_fill_kernel, grid, dim3(256), 0, s, elts, C, n_chunks, out->chunk_off, out->ev,
                       out->val);
    return hipGetLastError();
}

void free_sparse_pool(SparsePool* sp) {
    if (sp->ev) (void)hipFree(sp->ev);
    if (sp->val) (void)hipFree(sp->val);
    if (sp->chunk_off) (void)hipFree(sp->chunk_off);
    *sp = SparsePool{};
}
int64_t part_size() { return kPartSize; }
int part_tile_trials() { return kTileMax; }

hipError_t build_part_layout(const int64_t* offsets, const uint32_t* ids, int64_t N, int64_t n_events, int64_t C,
                             int n_cu, hipStream_t s, PartLayout* out) {
    *out = PartLayout{};
    const int P = static_cast<int>((C + kPartSize - 1) / kPartSize);
    if (P < 1 || P > kMaxParts || N < 1) return hipSuccess;            // layout not used
    const int T = kTileMax;
    const int64_t n_tiles = (N + T - 1) / T;
    hipError_t e;
    int32_t* cnt = nullptr;
    int64_t* tsize = nullptr;
    if ((e = dev_alloc(reinterpret_cast<void**>(&cnt), sizeof(int32_t) * N * P, s)) != hipSuccess) return e;
    if ((e = dev_alloc(reinterpret_cast<void**>(&out->seg_rel),
                            sizeof(uint32_t) * (n_tiles * (static_cast<int64_t>(T) * P + 1)), s)) != hipSuccess)
        goto fail;
    if ((e = dev_alloc(reinterpret_cast<void**>(&tsize), sizeof(int64_t) * n_tiles, s)) != hipSuccess) goto fail;
    if ((e = dev_alloc(reinterpret_cast<void**>(&out->tile_start), sizeof(int64_t) * (n_tiles + 1), s)) !=
        hipSuccess)
        goto fail;
    {
        int64_t blocks = (N + 3) / 4;
        if (blocks > int64_t(n_cu) * 16) blocks = int64_t(n_cu) * 16;
        hipLaunchKernelGGL(part_count_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, offsets, ids, N,
                           P, cnt);
        if ((e = hipGetLastError()) != hipSuccess) goto fail;
        hipLaunchKernelGGL(tile_scan_kernel, dim3(static_cast<uint32_t>(n_tiles)), dim3(256), 0, s, cnt, N, P, T,
                           out->seg_rel, tsize);
        if ((e = hipGetLastError()) != hipSuccess) goto fail;
        std::vector<int64_t> h(n_tiles), st(n_tiles + 1);
        if ((e = hipMemcpyAsync(h.data(), tsize, sizeof(int64_t) * n_tiles, hipMemcpyDeviceToHost, s)) != hipSuccess)
            goto fail;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) goto fail;
        st[0] = 0;
        for (int64_t k = 0; k < n_tiles; ++k) {
            if (h[k] >= (int64_t(1) << 31)) {   // too large for 32-bit positions: keep the plain layout
                dev_free(cnt, s);
                dev_free(tsize, s);
                dev_free(out->seg_rel, s);
                dev_free(out->tile_start, s);
                (void)hipStreamSynchronize(s);
                *out = PartLayout{};
                return hipSuccess;
            }
            st[k + 1] = st[k] + ((h[k] + kTileAlign - 1) & ~int64_t(kTileAlign - 1));   // padded with sentinels
        }
        const int64_t total = st[n_tiles];
        if ((e = hipMemcpyAsync(out->tile_start, st.data(), sizeof(int64_t) * (n_tiles + 1), hipMemcpyHostToDevice,
                                s)) != hipSuccess)
            goto fail;
        if ((e = dev_alloc(reinterpret_cast<void**>(&out->pids), sizeof(uint32_t) * (total + kIdPad), s)) !=
            hipSuccess)
            goto fail;
        int64_t fb = (total + kIdPad + 255) / 256;
        if (fb > 8192) fb = 8192;
        hipLaunchKernelGGL(fill_u32_kernel, dim3(static_cast<uint32_t>(fb)), dim3(256), 0, s, out->pids, total + kIdPad,
                           kSentinel);
        if ((e = hipGetLastError()) != hipSuccess) goto fail;
        {
            // one 16-wave workgroup per CU (the stage fills LDS), over runs of kChunkTrials trials
            int64_t sb = n_tiles * ((T + kChunkTrials - 1) / kChunkTrials);
            if (sb > int64_t(n_cu)) sb = n_cu;
            hipLaunchKernelGGL(part_scatter_kernel, dim3(static_cast<uint32_t>(sb)), dim3(1024), 0, s, offsets, ids, N,
                               P, T, out->seg_rel, out->tile_start, out->pids);
        }
        if ((e = hipGetLastError()) != hipSuccess) goto fail;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) goto fail;
        (void)n_events;
        out->P = P;
        out->T = T;
        out->n_tiles = n_tiles;
        out->length = total;
        out->bytes = sizeof(uint32_t) * (total + kIdPad) + sizeof(uint32_t) * (n_tiles * (int64_t(T) * P + 1)) +
                     sizeof(int64_t) * (n_tiles + 1);
    }
    // temporaries go back to the library's device memory cache: no free waits for the device
    dev_free(cnt, s);
    dev_free(tsize, s);
    return hipSuccess;
fail:
    if (cnt) dev_free(cnt, s);
    if (tsize) dev_free(tsize, s);
    free_part_layout(out, s);
    (void)hipStreamSynchronize(s);
    return e;
}

void free_part_layout(PartLayout* L, hipStream_t s) {
    if (L->pids) dev_free(L->pids, s);
    if (L->seg_rel) dev_free(L->seg_rel, s);
    if (L->tile_start) dev_free(L->tile_start, s);
    *L = PartLayout{};
}

int64_t part_scratch_bytes(int64_t C, int P) {
    const int64_t n_sb = static_cast<int64_t>(P) * kBase32;
    return part_image_bytes(P) + sizeof(uint32_t) * n_sb + sizeof(double) * C + sizeof(double) * n_sb * kSuper + 256;
}

namespace {
struct PartScratch {
    uint8_t* img;
    uint32_t* sb_count;
    uint32_t* counter;
    double* stage;        // [n_sb][kSuper]: each superblock's nonzero o, packed, before compaction
    double* compact;      // [C]: the nonzero o at their global ranks (last: sized by C)
};
PartScratch carve_parts(void* scratch, int P) {
    char* p = static_cast<char*>(scratch);
    PartScratch r;
    r.img = reinterpret_cast<uint8_t*>(p);
    p += part_image_bytes(P);
    const int64_t n_sb = static_cast<int64_t>(P) * kBase32;
    r.sb_count = reinterpret_cast<uint32_t*>(p);
    p += sizeof(uint32_t) * n_sb;
    r.counter = reinterpret_cast<uint32_t*>(p);
    p += 256;
    r.stage = reinterpret_cast<double*>(p);
    p += sizeof(double) * n_sb * kSuper;
    r.compact = reinterpret_cast<double*>(p);
    return r;
}
}  // namespace

double* part_compact_values(void* part_scratch, int P) { return carve_parts(part_scratch, P).compact; }
uint32_t* part_superblock_counts(void* part_scratch, int P) { return carve_parts(part_scratch, P).sb_count; }

// ---------------------------------------------------------------------------
// per-event net losses (the cumulative form of the aggregate terms)
// ---------------------------------------------------------------------------

namespace {

constexpr int kProbeShift = 5;                  // 32 catalogue events per probe word
constexpr int kNetsThreads = 1024;              // one workgroup per CU: its waves share the coarse map
constexpr int kNetsStageBytes = 37 * 1024;     // the waves' stage and flag rows
constexpr int kCoarseBytes = 160 * 1024 - kNetsStageBytes;   // LDS left for the coarse map

// value moved across lanes by a DPP control; lanes without a source get 0
template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), kCtrl, kRowMask, 0xF, false));
}
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t b = __double_as_longlong(v);
    const uint32_t lo = dpp_u32<kCtrl, kRowMask>(static_cast<uint32_t>(b));
    const uint32_t hi = dpp_u32<kCtrl, kRowMask>(static_cast<uint32_t>(b >> 32));
    return __longlong_as_double(static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo));
}
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int lane) {
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v)), lane);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v >> 32)), lane);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    return __longlong_as_double(static_cast<int64_t>(readlane_u64(static_cast<uint64_t>(__double_as_longlong(v)), lane)));
}

// One stage of a segmented double-double scan: (f, h, l) becomes
// left (+) self, where a lane that starts a segment (f set) keeps its sum.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ void seg_stage(uint32_t& f, double& h, double& l) {
    const uint32_t uf = dpp_u32<kCtrl, kRowMask>(f);
    const double uh = dpp_f64<kCtrl, kRowMask>(h), ul = dpp_f64<kCtrl, kRowMask>(l);
    double mh = h, ml = l;
    dd_merge(mh, ml, uh, ul);
    if (!f) {
        h = mh;
        l = ml;
        f = uf;
    }
}
// inclusive over the wave: row shifts 1, 2, 4, 8, then row broadcasts 15, 31
__device__ __forceinline__ void wave_seg_scan_dd(uint32_t& f, double& h, double& l) {
    seg_stage<0x111, 0xF>(f, h, l);
    seg_stage<0x112, 0xF>(f, h, l);
    seg_stage<0x114, 0xF>(f, h, l);
    seg_stage<0x118, 0xF>(f, h, l);
    seg_stage<0x142, 0xA>(f, h, l);
    seg_stage<0x143, 0xC>(f, h, l);
}

// smallest t in [lo, hi] with offsets[t] >= target, given offsets[hi] >=
// target; a 64-way search, all arguments uniform over the wave
__device__ int64_t first_trial_at(const int64_t* __restrict__ offsets, int64_t lo, int64_t hi, int64_t target,
                                  int lane) {
    while (hi - lo >= 64) {
        const int64_t step = (hi - lo) / 64;
        const uint64_t m = __ballot(offsets[lo + lane * step] >= target);   // index <= hi - step
        if (m == 0) {
            lo = lo + 63 * step + 1;
        } else {
            const int f = __builtin_ctzll(m);
            const int64_t nlo = f > 0 ? lo + (f - 1) * step + 1 : lo;
            hi = lo + f * step;
            lo = nlo;
        }
    }
    const int64_t idx = lo + lane;
    const uint64_t m = __ballot(idx <= hi && offsets[idx] >= target);
    return lo + __builtin_ctzll(m);
}

// probe word per 32 catalogue events: the bitmap bits (low half) and the
// rank of the word's first event among the nonzero ones (high half), built
// from the part images
__global__ __launch_bounds__(256) void probe_table_kernel(const uint8_t* __restrict__ img, int64_t n_words,
                                                          uint64_t* __restrict__ probe) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_words) return;
    constexpr int kShift = kPartShift - kProbeShift;                    // probe words per part
    const uint8_t* base = img + (i >> kShift) * kImgBytes;
    const uint32_t j = static_cast<uint32_t>(i & ((int64_t(1) << kShift) - 1));
    const uint32_t* bm32 = reinterpret_cast<const uint32_t*>(base);
    const uint16_t* r16 = reinterpret_cast<const uint16_t*>(base + int64_t(kWords) * 8);
    const uint32_t* b32 = reinterpret_cast<const uint32_t*>(base + int64_t(kWords) * 8 + int64_t(kRank16) * 2);
    uint32_t rank = b32[j >> 7] + r16[j >> 2];       // superblock base, 128-event offset
    for (uint32_t k = j & ~3u; k < j; ++k) rank += __builtin_popcount(bm32[k]);
    probe[i] = (static_cast<uint64_t>(rank) << 32) | bm32[j];
}

// coarse map: bit i is set when any of events [i << cshift, (i + 1) << cshift)
// has a nonzero loss; one thread per 32-bit word, from the probe words' bits
__global__ __launch_bounds__(256) void coarse_map_kernel(const uint64_t* __restrict__ probe, int64_t n_words,
                                                         int cshift, int64_t n_cw, uint32_t* __restrict__ coarse) {
    const int64_t cw = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (cw >= n_cw) return;
    uint32_t out = 0;
    for (int k = 0; k < 32; ++k) {
        const int64_t s0 = (cw * 32 + k) << cshift;                   // first event of the group
        uint32_t any = 0;
        if (cshift >= kProbeShift) {
            const int64_t w0 = s0 >> kProbeShift, nw = int64_t(1) << (cshift - kProbeShift);
            for (int64_t w = w0; w < w0 + nw && w < n_words; ++w) any |= static_cast<uint32_t>(probe[w]);
        } else if ((s0 >> kProbeShift) < n_words) {
            const uint32_t bits = static_cast<uint32_t>(probe[s0 >> kProbeShift]);
            const uint32_t width = 1u << cshift;
            const uint32_t mask = (width >= 32u ? ~0u : ((1u << width) - 1u)) << (s0 & 31);
            any = bits & mask;
        }
        out |= (any != 0u ? 1u : 0u) << k;
    }
    coarse[cw] = out;
}

// The layer's trials are split into one contiguous run per wave (event
// shares rounded to trial starts), and each wave streams its run's IDs in
// steps of 64 kE positions in time order, kE consecutive positions per lane
// (16-byte loads, the next step's issued before this step's work).  o(E) is
// 0 unless E's bit is set in its probe word, else compact[rank + bits below]
// -- an 8-byte probe and one more load per nonzero loss, both from tables
// that stay in L2.  L2 serves these random requests at a bounded rate, so the
// workgroup's 16 waves first test a coarse map in LDS (one bit per 2^cshift
// events, set when any of them has a loss) and probe L2 only for events
// whose bit is set.  Trial starts (held one per lane and marked in a
// per-wave LDS bit row) reset a segmented double-double scan: each event's
// running total S_d (the lane's own prefix, the scan of the lanes before it,
// the carry of earlier steps) is rounded once; A_d = clamp(S_d; AggR, AggL)
// and the net is A_d - A_{d-1}, with A_{d-1} = A_0 = clamp(0; AggR, AggL)
// for a trial's first event, so a trial's nets telescope to its year loss
// minus A_0.  A lane forms its kE nets in registers (A of the position before
// its first one comes from the lane below); the nets go through a per-wave
// LDS stage, half a step at a time, and out in non-temporal stores of 64
// consecutive values.  With kStride the kernel writes, instead of nets, the
// running total S_d of every position d = 64b + 63 to slot b of `nets` (the
// stride checkpoints of the forward pass) and needs no stage.  Eight events
// per lane spread the wave scan over twice the events of four.
template <int kE, bool kStride = false>
__global__ __launch_bounds__(kNetsThreads) void event_nets_kernel(const int64_t* __restrict__ offsets,
                                                                  const uint32_t* __restrict__ ids,
                                                                  const uint64_t* __restrict__ probe,
                                                                  const uint32_t* __restrict__ gcoarse, int cshift,
                                                                  int64_t n_cw, const double* __restrict__ compact,
                                                                  LayerArgs L, double* __restrict__ nets) {
    static_assert(kE == 4 || kE == 8, "four or eight events per lane");
    static_assert(64 % kE == 0, "stride slots are lanes' last events when kE divides 64");
    constexpr int kW = 64 * kE;                                        // positions per step
    static_assert(kW <= kIdPad, "a step may read up to kW - 1 IDs past the table's end");
    constexpr int kRow = 32 * (kE + 1);        // half a step's nets, one pad slot per lane
    static_assert(kNetsStageBytes >= (kNetsThreads / 64) * (kRow * 8 + kW / 8), "stage rows fit their LDS share");
    __shared__ double stage[kNetsThreads / 64][kStride ? 1 : kRow];
    __shared__ uint32_t flag_rows[kNetsThreads / 64][kW / 32];          // bit i: a trial starts at c + i
    extern __shared__ uint32_t coarse[];                               // [n_cw]
    // the coarse map, before any wave can leave (the only workgroup barrier)
    for (int64_t i = threadIdx.x; i < n_cw; i += blockDim.x) coarse[i] = gcoarse[i];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    double* st = stage[threadIdx.x >> 6];
    uint32_t* fl = flag_rows[threadIdx.x >> 6];
    const int64_t w = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t n_w = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
    const int64_t t0 = L.trial_begin, t1 = L.trial_begin + L.trial_count;
    const int64_t ev0 = offsets[t0];
    const int64_t tot = offsets[t1] - ev0;
    const int64_t k0 = first_trial_at(offsets, t0, t1, ev0 + tot * w / n_w, lane);
    const int64_t k1 = first_trial_at(offsets, t0, t1, ev0 + tot * (w + 1) / n_w, lane);
    if (k0 >= k1) return;
    const int64_t P0 = offsets[k0], P1 = offsets[k1];
    if (P0 >= P1) return;
    const double A0 = apply_terms(0.0, L.aggR, L.aggL);
    if (lane < kW / 32) fl[lane] = 0;
    int64_t kb = k0;                                                   // trial starts held: kb .. kb + 63
    int64_t bnd = kb + lane < k1 ? offsets[kb + lane] : INT64_MAX;
    const int64_t c0 = P0 & ~int64_t(kE - 1);                          // 16-byte and lane aligned
    u32x4 nxt[kE / 4];
#pragma unroll
    for (int u = 0; u < kE / 4; ++u)
        nxt[u] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(ids + c0 + lane * kE + 4 * u));
    double ch = 0.0, cl = 0.0;       // running total of the segment open at the step's start
    double a_prev = A0;              // A of the position before the step
    for (int64_t c = c0; c < P1; c += kW) {
        u32x4 cur[kE / 4];
#pragma unroll
        for (int u = 0; u < kE / 4; ++u) cur[u] = nxt[u];
        if (c + kW < P1) {
#pragma unroll
            for (int u = 0; u < kE / 4; ++u)
                nxt[u] = __builtin_nontemporal_load(
                    reinterpret_cast<const u32x4*>(ids + c + kW + lane * kE + 4 * u));
        }
        // mark the trial starts inside [c, c + kW)
        for (;;) {
            if (bnd >= c && bnd < c + kW) {
                const uint32_t i = static_cast<uint32_t>(bnd - c);
                atomicOr(&fl[i >> 5], 1u << (i & 31u));
            }
            if (static_cast<int64_t>(readlane_u64(static_cast<uint64_t>(bnd), 63)) >= c + kW) break;
            kb += 64;
            bnd = kb + lane < k1 ? offsets[kb + lane] : INT64_MAX;
        }
        __builtin_amdgcn_wave_barrier();
        uint32_t fq[kE];
        {
            const uint32_t fb = fl[(lane * kE) >> 5] >> ((lane * kE) & 31);
#pragma unroll
            for (int q = 0; q < kE; ++q) fq[q] = (fb >> q) & 1u;
        }
        const int64_t pos = c + lane * kE;
        uint32_t E[kE];
        bool ok[kE];
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            ok[q] = pos + q >= P0 && pos + q < P1;
            E[q] = ok[q] ? cur[q >> 2][q & 3] : 0u;
        }
        // the L2 probe only where the coarse map says the event's group has a loss
        uint64_t pw[kE];
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const uint32_t cb = E[q] >> cshift;
            pw[q] = 0;
            if (ok[q] && ((coarse[cb >> 5] >> (cb & 31u)) & 1u)) pw[q] = probe[E[q] >> kProbeShift];
        }
        double oq[kE];
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const uint32_t bits = static_cast<uint32_t>(pw[q]);
            const uint32_t bi = E[q] & 31u;
            oq[q] = 0.0;
            if (ok[q] && ((bits >> bi) & 1u)) {
                const uint32_t below = bi ? (~0u >> (32u - bi)) : 0u;
                oq[q] = compact[static_cast<uint32_t>(pw[q] >> 32) + __builtin_popcount(bits & below)];
            }
        }
        // the lane's total since its last trial start (all of it if none)
        uint32_t sf = 0;
        double h = 0.0, l = 0.0;
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            if (fq[q]) {
                h = 0.0;
                l = 0.0;
            }
            dd_add(h, l, oq[q]);
            sf |= fq[q];
        }
        if (lane == 0 && !sf) dd_merge(h, l, ch, cl);              // the open segment's carry
        double sh = h, sl = l;
        wave_seg_scan_dd(sf, sh, sl);
        if constexpr (kStride) {
            // a lane's first position is a multiple of kE, and kE divides 64, so
            // each 64b + 63 is some lane's last event, where the running total is
            // that lane's inclusive scan
            if (ok[kE - 1] && ((pos + kE - 1) & 63) == 63) nets[(pos + kE - 1) >> 6] = sh + sl;
        } else {
            // the open segment's total before this lane's first event, then the
            // running totals again, event by event, and A of each position
            double rh = __shfl_up(sh, 1, 64), rl = __shfl_up(sl, 1, 64);
            if (lane == 0) {
                rh = ch;
                rl = cl;
            }
            double A[kE];
#pragma unroll
            for (int q = 0; q < kE; ++q) {
                if (fq[q]) {
                    rh = 0.0;
                    rl = 0.0;
                }
                dd_add(rh, rl, oq[q]);
                A[q] = apply_terms(rh + rl, L.aggR, L.aggL);
            }
            // A of the position before each: A_0 before a trial's first event,
            // the lane below's last A before this lane's first, a_prev before the step's
            double before = __shfl_up(A[kE - 1], 1, 64);
            if (lane == 0) before = a_prev;
            double net[kE];
#pragma unroll
            for (int q = 0; q < kE; ++q) net[q] = A[q] - (fq[q] ? A0 : (q == 0 ? before : A[q - 1]));
            a_prev = readlane_f64(A[kE - 1], 63);
            // half a step at a time: lanes [32 hf, 32 hf + 32) hold positions
            // [kW/2 hf, kW/2 (hf + 1)); position i of the half sits at i + i / kE
#pragma unroll
            for (int hf = 0; hf < 2; ++hf) {
                if ((lane >> 5) == hf) {
#pragma unroll
                    for (int q = 0; q < kE; ++q) st[(lane & 31) * (kE + 1) + q] = net[q];
                }
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int r = 0; r < kE / 2; ++r) {
                    const int i = r * 64 + lane;
                    const int64_t p = c + hf * (kW / 2) + i;
                    const double v = st[i + i / kE];
                    if (p >= P0 && p < P1) __builtin_nontemporal_store(v, nets + (p - ev0));
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        ch = readlane_f64(sh, 63);
        cl = readlane_f64(sl, 63);
        __builtin_amdgcn_wave_barrier();
        if (lane < kW / 32) fl[lane] = 0;
    }
}

}  // namespace

int part_count(int64_t C) { return static_cast<int>((C + kPartSize - 1) / kPartSize); }

int64_t probe_table_bytes(int64_t C) {
    // probe words, then the coarse map (at most kCoarseBytes)
    return static_cast<int64_t>(sizeof(uint64_t)) * ((C + (1 << kProbeShift) - 1) >> kProbeShift) + 256 +
           kCoarseBytes;
}

namespace {

hipError_t launch_nets_or_stride(const int64_t* offsets, const uint32_t* ids, const void* part_scratch, int P,
                                 int64_t C, uint64_t* probe, const LayerArgs& L, double* out, bool stride, int n_cu,
                                 hipStream_t s) {
    if (L.trial_count <= 0) return hipSuccess;
    PartScratch ps = carve_parts(const_cast<void*>(part_scratch), P);
    const int64_t n_words = (C + (1 << kProbeShift) - 1) >> kProbeShift;
    hipLaunchKernelGGL(probe_table_kernel, dim3(static_cast<uint32_t>((n_words + 255) / 256)), dim3(256), 0, s,
                       ps.img, n_words, probe);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the finest coarse map that fits: 2^cshift events per bit
    int cshift = 0;
    while ((((C + (int64_t(1) << cshift) - 1) >> cshift) + 31) / 32 * 4 > kCoarseBytes) ++cshift;
    const int64_t n_cw = (((C + (int64_t(1) << cshift) - 1) >> cshift) + 31) / 32;
    uint32_t* coarse = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(probe) + sizeof(uint64_t) * n_words + 256);
    hipLaunchKernelGGL(coarse_map_kernel, dim3(static_cast<uint32_t>((n_cw + 255) / 256)), dim3(256), 0, s, probe,
                       n_words, cshift, n_cw, coarse);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const size_t lds = sizeof(uint32_t) * static_cast<size_t>(n_cw);
    int per_cu = 0;
    if ((stride ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, event_nets_kernel<8, true>, kNetsThreads, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, event_nets_kernel<8, false>, kNetsThreads,
                                                                lds)) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int64_t blocks = (L.trial_count + kNetsThreads / 64 - 1) / (kNetsThreads / 64);
    const int64_t cap = static_cast<int64_t>(n_cu) * per_cu;
    if (blocks > cap) blocks = cap;
    if (stride)
        hipLaunchKernelGGL((event_nets_kernel<8, true>), dim3(static_cast<uint32_t>(blocks)), dim3(kNetsThreads), lds,
                           s, offsets, ids, probe, coarse, cshift, n_cw, ps.compact, L, out);
    else
        hipLaunchKernelGGL((event_nets_kernel<8, false>), dim3(static_cast<uint32_t>(blocks)), dim3(kNetsThreads), lds,
                           s, offsets, ids, probe, coarse, cshift, n_cw, ps.compact, L, out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_event_nets(const int64_t* offsets, const uint32_t* ids, const void* part_scratch, int P,
                             int64_t C, uint64_t* probe, const LayerArgs& L, double* nets, int n_cu, hipStream_t s) {
    return launch_nets_or_stride(offsets, ids, part_scratch, P, C, probe, L, nets, false, n_cu, s);
}

hipError_t launch_stride_checkpoints(const int64_t* offsets, const uint32_t* ids, const void* part_scratch, int P,
                                     int64_t C, uint64_t* probe, const LayerArgs& L, double* stride, int n_cu,
                                     hipStream_t s) {
    return launch_nets_or_stride(offsets, ids, part_scratch, P, C, probe, L, stride, true, n_cu, s);
}

hipError_t launch_part_fold(const double* o, int64_t C, int P, void* scratch, hipStream_t s, bool with_ranks) {
    PartScratch ps = carve_parts(scratch, P);
    const int64_t n_sb = static_cast<int64_t>(P) * kBase32;
    hipError_t e;
    hipLaunchKernelGGL(part_image_kernel, dim3(static_cast<uint32_t>(n_sb)), dim3(256), 0, s, o, C, ps.img,
                       ps.sb_count, int64_t(0), int64_t(0), int64_t(0));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (!with_ranks) return hipSuccess;
    hipLaunchKernelGGL(superblock_scan_kernel, dim3(1), dim3(1024), 0, s, ps.sb_count, n_sb, ps.img, int64_t(0));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(compact_kernel, dim3(static_cast<uint32_t>(n_sb)), dim3(256), 0, s, o, C, ps.img, ps.compact,
                       int64_t(0), int64_t(0));
    return hipGetLastError();
}

hipError_t launch_fold_parts(const SparsePool& sp, int64_t C, const LayerArgs& L, const LayerArgs* L_dev, double* o,
                             int P, void* scratch, hipStream_t s) {
    PartScratch ps = carve_parts(scratch, P);
    const int64_t n_sb = static_cast<int64_t>(P) * kBase32;
    hipError_t e;
    if (L_dev)
        hipLaunchKernelGGL(fold_image_dev_kernel, dim3(static_cast<uint32_t>(n_sb)), dim3(256), 0, s, sp, C, L_dev,
                           o, ps.img, ps.sb_count, ps.stage);
    else
        hipLaunchKernelGGL(fold_image_kernel, dim3(static_cast<uint32_t>(n_sb)), dim3(256), 0, s, sp, C, L, o,
                           ps.img, ps.sb_count, ps.stage);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(compact_stage_kernel, dim3(static_cast<uint32_t>(n_sb)), dim3(256), 0, s, ps.stage,
                       ps.sb_count, ps.img, ps.compact);
    return hipGetLastError();
}

hipError_t launch_part_pass(const PartLayout& lay, int64_t N, const LayerArgs& L, void* scratch, double* ylt,
                            double* S, int n_cu, hipStream_t s, int lpt) {
    if (L.trial_count <= 0) return hipSuccess;
    const int P = lay.P;
    PartScratch ps = carve_parts(scratch, P);
    hipError_t e;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, s, ps.counter, int64_t(1), 0u);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    PartPassArgs a{};
    a.pids = lay.pids;
    a.seg_rel = lay.seg_rel;
    a.tile_start = lay.tile_start;
    a.img = ps.img;
    a.compact = ps.compact;
    a.N = N;
    a.P = P;
    a.T = lay.T;
    a.t_lo = L.trial_begin;
    a.t_hi = L.trial_begin + L.trial_count;
    a.first_tile = L.trial_begin / lay.T;
    a.last_tile = (a.t_hi + lay.T - 1) / lay.T;
    a.aggR = L.aggR;
    a.aggL = L.aggL;
    a.ylt = ylt;
    a.S = S;
    a.tile_counter = ps.counter;
    int64_t grid = a.last_tile - a.first_tile;
    if (grid > int64_t(n_cu) * 2) grid = int64_t(n_cu) * 2;
    return launch_part_pass_lpt(lpt, static_cast<int>(grid), a, s);
}

}  // namespace ara

namespace ara {

hipError_t launch_part_adjoint(const PartLayout& lay, int64_t N, const LayerArgs& L, void* part_scratch,
                               const double* S, const double* ylt, const TailStats* tail, uint64_t* w_mean,
                               uint64_t* w_tvar, int n_cu, hipStream_t s) {
    if (L.trial_count <= 0) return hipSuccess;
    PartScratch ps = carve_parts(part_scratch, lay.P);
    hipError_t e;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, s, ps.counter, int64_t(1), 0u);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    PartAdjArgs a{};
    a.pids = lay.pids;
    a.seg_rel = lay.seg_rel;
    a.tile_start = lay.tile_start;
    a.img = ps.img;
    a.N = N;
    a.P = lay.P;
    a.T = lay.T;
    a.t_lo = L.trial_begin;
    a.t_hi = L.trial_begin + L.trial_count;
    a.first_tile = L.trial_begin / lay.T;
    a.last_tile = (a.t_hi + lay.T - 1) / lay.T;
    a.aggR = L.aggR;
    a.aggL = L.aggL;
    a.S = S;
    a.ylt = ylt;
    a.tail = tail;
    a.w_mean = w_mean;
    a.w_tvar = w_tvar;
    a.tile_counter = ps.counter;
    a.sb_count = ps.sb_count;
    if (lay.length < (int64_t(1) << 32)) {
        // one workgroup per CU, a multiple of the XCD count (see xcd_adjoint_kernel)
        int64_t grid = int64_t(n_cu);
        grid -= grid % kXcds;
        if (grid < kXcds) grid = kXcds;
        hipLaunchKernelGGL(xcd_adjoint_kernel, dim3(static_cast<uint32_t>(grid)), dim3(1024), 0, s, a, kXcds);
        return hipGetLastError();
    }
    int64_t grid = a.last_tile - a.first_tile;
    if (grid > int64_t(n_cu) * 2) grid = int64_t(n_cu) * 2;
    hipLaunchKernelGGL(part_adjoint_kernel, dim3(static_cast<uint32_t>(grid)), dim3(512), 0, s, a);
    return hipGetLastError();
}

}  // namespace ara

namespace ara {

int64_t batched_scratch_bytes(int64_t C, int P, int n_layers, int64_t n_items, int64_t n_elts_total) {
    const int64_t n_sb = static_cast<int64_t>(P) * kBase32;
    int64_t b = 0;
    b += sizeof(double) * C * n_layers;                  // o
    b += sizeof(double) * C * n_layers;                  // compact
    b += part_image_bytes(P) * n_layers;                 // images
    b += sizeof(uint32_t) * n_sb * n_layers;             // superblock counts
    b += 256;                                            // counter
    b += sizeof(int2) * n_items + 256;
    b += sizeof(BatchLayerDesc) * n_layers + sizeof(BatchFoldDesc) * n_layers + 512;
    b += (sizeof(int32_t) + 2 * sizeof(double)) * n_elts_total + 512;
    return b;
}

BatchedScratch carve_batched(void* scratch, int64_t C, int P, int n_layers, int64_t n_items, int64_t n_elts_total) {
    char* p = static_cast<char*>(scratch);
    const int64_t n_sb = static_cast<int64_t>(P) * kBase32;
    BatchedScratch r;
    r.o = reinterpret_cast<double*>(p);
    p += sizeof(double) * C * n_layers;
    r.compact = reinterpret_cast<double*>(p);
    p += sizeof(double) * C * n_layers;
    r.img = reinterpret_cast<uint8_t*>(p);
    p += part_image_bytes(P) * n_layers;
    r.sb_count = reinterpret_cast<uint32_t*>(p);
    p += sizeof(uint32_t) * n_sb * n_layers;
    r.counter = reinterpret_cast<uint32_t*>(p);
    p += 256;
    r.items = reinterpret_cast<int2*>(p);
    p += sizeof(int2) * n_items + 256;
    r.layers = reinterpret_cast<BatchLayerDesc*>(p);
    p += sizeof(BatchLayerDesc) * n_layers;
    r.fold = reinterpret_cast<BatchFoldDesc*>(p);
    p += sizeof(BatchFoldDesc) * n_layers + 512;
    r.R = reinterpret_cast<double*>(p);
    p += sizeof(double) * n_elts_total;
    r.Lim = reinterpret_cast<double*>(p);
    p += sizeof(double) * n_elts_total;
    r.idx = reinterpret_cast<int32_t*>(p);
    return r;
}

hipError_t launch_batched(const PartLayout& lay, int64_t N, int64_t C, const double* elts, int n_layers,
                          const BatchedScratch& b, int64_t n_items, double* ylt, int n_cu, hipStream_t s,
                          hipEvent_t pass_start, hipEvent_t pass_stop, int lpt) {
    hipError_t e;
    const int P = lay.P;
    const int64_t n_sb = static_cast<int64_t>(P) * kBase32;
    const int64_t img_stride = part_image_bytes(P);
    hipLaunchKernelGGL(batched_fold_kernel, dim3(static_cast<uint32_t>((C + 255) / 256), n_layers), dim3(256), 0, s,
                       elts, C, b.fold, b.idx, b.R, b.Lim, b.o);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(part_image_kernel, dim3(static_cast<uint32_t>(n_sb), n_layers), dim3(256), 0, s, b.o, C, b.img,
                       b.sb_count, C, img_stride, n_sb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(superblock_scan_kernel, dim3(1, n_layers), dim3(1024), 0, s, b.sb_count, n_sb, b.img,
                       img_stride);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(compact_kernel, dim3(static_cast<uint32_t>(n_sb), n_layers), dim3(256), 0, s, b.o, C, b.img,
                       b.compact, C, img_stride);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, s, b.counter, int64_t(1), 0u);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    BatchedPassArgs a{};
    a.pids = lay.pids;
    a.seg_rel = lay.seg_rel;
    a.tile_start = lay.tile_start;
    a.img = b.img;
    a.img_stride = img_stride;
    a.compact = b.compact;
    a.C = C;
    a.N = N;
    a.P = P;
    a.T = lay.T;
    a.items = b.items;
    a.n_items = static_cast<int32_t>(n_items);
    a.layers = b.layers;
    a.ylt = ylt;
    a.item_counter = b.counter;
    int64_t grid = n_items < int64_t(n_cu) * 2 ? n_items : int64_t(n_cu) * 2;
    if (grid < 1) grid = 1;
    if (pass_start && (e = hipEventRecord(pass_start, s)) != hipSuccess) return e;
    if ((e = launch_batched_pass_lpt(lpt, static_cast<int>(grid), a, s)) != hipSuccess) return e;
    if (pass_stop && (e = hipEventRecord(pass_stop, s)) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace ara

namespace ara {

hipError_t launch_xcd_pass(const PartLayout& lay, int64_t N, int64_t C, const LayerArgs& L, void* part_scratch,
                           double* partials, int n_cu, hipStream_t s) {
    if (L.trial_count <= 0) return hipSuccess;
    const int P = lay.P;
    PartScratch ps = carve_parts(part_scratch, P);
    XcdPassArgs a{};
    a.pids = lay.pids;
    a.seg_rel = lay.seg_rel;
    a.tile_start = lay.tile_start;
    a.img = ps.img;
    a.compact = ps.compact;
    a.C = C;
    a.N = N;
    a.P = P;
    a.T = lay.T;
    a.t_lo = L.trial_begin;
    a.t_hi = L.trial_begin + L.trial_count;
    a.first_tile = L.trial_begin / lay.T;
    a.last_tile = (a.t_hi + lay.T - 1) / lay.T;
    a.part_hi = partials;
    a.part_lo = partials + static_cast<int64_t>(P) * L.trial_count;
    a.pad = lay.pids + lay.length;
    a.n_xcd = kXcds;
    // one 1024-thread workgroup per CU (its LDS holds the part image and the
    // loss cache), a multiple of the XCD count so every XCD gets the same share
    int64_t grid = int64_t(n_cu);
    grid -= grid % kXcds;
    if (grid < kXcds) grid = kXcds;
    hipLaunchKernelGGL(xcd_pass_kernel, dim3(static_cast<uint32_t>(grid)), dim3(1024), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_xcd_combine(const PartLayout& lay, const LayerArgs& L, const LayerArgs* L_dev,
                              const double* partials, double* ylt, double* S, hipStream_t s) {
    if (L.trial_count <= 0) return hipSuccess;
    const int P = lay.P;
    const int64_t blocks = (L.trial_count + 255) / 256;
    hipLaunchKernelGGL(xcd_combine_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, partials,
                       partials + static_cast<int64_t>(P) * L.trial_count, P, L.trial_count, L.aggR, L.aggL, L_dev, ylt,
                       S);
    return hipGetLastError();
}

}  // namespace ara
