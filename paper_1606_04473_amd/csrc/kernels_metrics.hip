// Risk metrics from a Year Loss Table: mean, PML_p, TVaR_p.
//
// Year losses are >= 0, so their IEEE-754 bit patterns order like their
// values when read as uint64.  PML_p (the m-th largest) is found by a radix
// select over those patterns with 12/12/12/12/12/4-bit digits, each pass a
// privatised LDS histogram of the values that match the prefix chosen so
// far.  The digit of a pass is chosen at the start of the next pass by every
// workgroup from the previous histogram (the same data, so the same choice),
// which saves a launch per pass; three histograms rotate so that the one
// being cleared is never read or written in the same pass.  All requested
// probabilities advance together.  For ara_risk_metrics (and the adjoint's
// tail statistics) the first two passes run over all values; then one pass sums the values above each 24-bit
// prefix and collects the keys inside it (a handful, unless many losses tie),
// and a single workgroup finishes the selection over those candidates: up to
// 256 of them are ranked directly against each other, more go through the
// last four digit passes.  Each launch costs about 9 us here, whatever its data, so
// that cuts nine launches to five.  The scratch is kept between calls and each
// call leaves it ready for the next (its candidate pass clears the first
// histogram, its last kernel the error flag), so a call on a reused scratch
// skips the init kernel: four launches.  TVaR_p = (sum of the values above v +
// (m - c_gt) v) / m, with v = PML_p and c_gt the count above it.  Sums are
// double-double, reduced in a fixed order (deterministic), and the product
// (m - c_gt) v is added exactly via fma.
#include "ara_internal.hpp"

namespace ara {

namespace {

constexpr int kSumBlocks = 512;
static_assert(kSumBlocks % 256 == 0, "the finishing workgroup holds kSumBlocks / 256 partials per thread");
constexpr int kBins = 4096;
constexpr int kPasses = 6;
constexpr int kMaxProbs = 4;   // 4 x 16 KB histograms fit the 64 KB dynamic-LDS default
constexpr int kDirect = 256;   // candidates ranked directly (all pairs) instead of by radix digits
// Workgroup sizes of the two histogram passes.  Each workgroup adds its
// nonzero bins to the global histogram with device atomics, and those on one
// bin serialise (in the first pass the values crowd into the few bins of
// their exponents), so fewer, larger workgroups wait less: 45.7 against
// 51.5 us for 1M losses and two probabilities with 256 threads in both.
constexpr int kHist0Threads = 1024;
constexpr int kHist1Threads = 1024;
__constant__ int kShift[kPasses] = {52, 40, 28, 16, 4, 0};
__constant__ int kBits[kPasses] = {12, 12, 12, 12, 12, 4};

struct SelState {
    uint64_t prefix;
    uint64_t mask;
    int64_t k;      // rank still to find inside the current prefix (1-based)
    int64_t m;
};

struct Scratch {
    double* part_hi;      // [kMaxProbs + 1][kSumBlocks]
    double* part_lo;
    int64_t* part_cnt;
    uint32_t* hist;       // [3][kMaxProbs][kBins]: pass k fills hist[k % 3]
    SelState* st;         // [2][kMaxProbs]: the state pass k uses is st[k & 1] (pass 0: st[0])
    uint32_t* flag;
    uint32_t* ccount;     // [kMaxProbs] candidates collected per probability
    uint64_t* cand;       // [n_probs][n] keys inside each probability's 24-bit prefix
};

constexpr int64_t kHistStride = int64_t(kMaxProbs) * kBins;   // one rotating histogram

constexpr int64_t kCandAlign = 256;

constexpr int64_t base_bytes() {
    return static_cast<int64_t>(kMaxProbs + 1) * kSumBlocks * (2 * sizeof(double) + sizeof(int64_t)) +
           3 * kHistStride * sizeof(uint32_t) + 2 * kMaxProbs * sizeof(SelState) + 64;
}

// Scratch of the allocation-free entry point: the fixed block plus candidate
// keys for up to kMaxProbs x kStaticTrials year losses (32.2 MiB).  A static
// device array, so each device the library runs on holds its own copy until
// the process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (metrics_noalloc_scratch).
constexpr int64_t kStaticTrials = int64_t(1) << 20;
constexpr int64_t kStaticBytes =
    (base_bytes() + kCandAlign - 1) / kCandAlign * kCandAlign + kMaxProbs * kStaticTrials * int64_t(sizeof(uint64_t));
static __device__ __align__(256) uint8_t scratch[kStaticBytes];

Scratch carve(void* base, int n_probs) {
    (void)n_probs;
    char* p = static_cast<char*>(base);
    char* const start = p;
    Scratch s;
    const int64_t np = static_cast<int64_t>(kMaxProbs + 1) * kSumBlocks;
    s.part_hi = reinterpret_cast<double*>(p);
    p += np * sizeof(double);
    s.part_lo = reinterpret_cast<double*>(p);
    p += np * sizeof(double);
    s.part_cnt = reinterpret_cast<int64_t*>(p);
    p += np * sizeof(int64_t);
    s.hist = reinterpret_cast<uint32_t*>(p);
    p += 3 * kHistStride * sizeof(uint32_t);
    s.st = reinterpret_cast<SelState*>(p);
    p += 2 * kMaxProbs * sizeof(SelState);
    s.flag = reinterpret_cast<uint32_t*>(p);
    s.ccount = reinterpret_cast<uint32_t*>(p + 16);
    s.cand = reinterpret_cast<uint64_t*>(start + (base_bytes() + kCandAlign - 1) / kCandAlign * kCandAlign);
    return s;
}

__device__ __forceinline__ uint64_t key_of(double x) {
    // +0.0 for -0.0 so that zero losses of either sign rank lowest
    return __double_as_longlong(x + 0.0);
}

// block-wide double-double reduction; result valid in thread 0
__device__ __forceinline__ void block_reduce_dd(double& hi, double& lo, int64_t& cnt) {
    __shared__ double sh[16], sl[16];              // up to 1024 threads
    __shared__ int64_t sc[16];
    group_reduce_dd(hi, lo, kWave);
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, kWave);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[w] = hi;
        sl[w] = lo;
        sc[w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        hi = sh[0];
        lo = sl[0];
        cnt = sc[0];
        const int nw = blockDim.x >> 6;
        for (int i = 1; i < nw; ++i) {
            dd_merge(hi, lo, sh[i], sl[i]);
            cnt += sc[i];
        }
    }
}

struct MArgs {
    int64_t m[kMaxProbs];
};

// Choose the digit of `pass` for one probability from that pass's histogram
// h, starting from the state st the pass used: the digit (from the top)
// whose bin holds the k-th largest remaining value.  Every thread of the
// 256-thread workgroup calls it and gets the new state.
__device__ SelState choose_digit(const uint32_t* __restrict__ h, SelState st, int pass) {
    __shared__ uint64_t scan[256];
    __shared__ SelState out;
    const int nb = 1 << kBits[pass];
    const int per = (nb + 255) / 256;                    // 16 (12-bit digits) or 1 (the last, 4-bit)
    // thread i owns bins [nb - per (i+1), nb - per i): thread 0 the largest digits
    const int t = threadIdx.x;
    const bool owner = t < 256;                           // larger workgroups: the rest wait at the barriers
    const int hiBin = nb - per * (owner ? t : 0);
    const int loBin = hiBin - per;
    uint32_t cnt[16];
    if (!owner) {
#pragma unroll
        for (int k = 0; k < 16; ++k) cnt[k] = 0;
    } else if (per == 16) {                               // 16 aligned bins: four 16-byte loads
        const u32x4* v = reinterpret_cast<const u32x4*>(h + loBin);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const u32x4 t = v[k];
            cnt[4 * k] = t.x;
            cnt[4 * k + 1] = t.y;
            cnt[4 * k + 2] = t.z;
            cnt[4 * k + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) cnt[k] = (k < per && loBin + k >= 0) ? h[loBin + k] : 0u;
    }
    uint64_t local = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) local += cnt[k];
    if (t == 0) out = st;                 // unchanged unless a bin is chosen (k beyond the count)
    if (owner) scan[t] = local;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint64_t add = owner && t >= off ? scan[t - off] : 0;
        __syncthreads();
        if (owner) scan[t] += add;
        __syncthreads();
    }
    const uint64_t incl = owner ? scan[t] : 0;
    const uint64_t excl = incl - local;
    const uint64_t k = static_cast<uint64_t>(st.k);
    if (owner && excl < k && k <= incl) {
        uint64_t cum = excl;
        for (int i = per - 1; i >= 0; --i) {              // from this thread's largest digit down
            const uint64_t c = cnt[i];
            if (cum + c >= k) {
                const int b = loBin + i;
                const int shift = kShift[pass];
                const uint64_t dmask = (uint64_t(1) << kBits[pass]) - 1;
                SelState r = st;
                r.k = static_cast<int64_t>(k - cum);
                r.prefix = st.prefix | (static_cast<uint64_t>(b) << shift);
                r.mask = st.mask | (dmask << shift);
                out = r;
                break;
            }
            cum += c;
        }
    }
    __syncthreads();
    const SelState r = out;
    __syncthreads();
    return r;
}

// resets the selection state and clears the first histogram (every
// probability's slot) with plain stores
__global__ void select_init_kernel(Scratch s, MArgs ma, int n_probs) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < n_probs) {
        s.st[tid].prefix = 0;
        s.st[tid].mask = 0;
        s.st[tid].k = ma.m[tid];
        s.st[tid].m = ma.m[tid];
    }
    if (tid == 0) *s.flag = 0;
    if (tid < kMaxProbs) s.ccount[tid] = 0;
    for (int64_t i = tid; i < kHistStride; i += gridDim.x * blockDim.x) s.hist[i] = 0;
}

// Pass `pass` of the radix select (and, in pass 0, the sum for the mean):
// finish the previous pass's digit choice, clear the histogram the next pass
// fills, and count this pass's digits of the values matching the prefix.
template <int kT>
__global__ __launch_bounds__(kT) void histogram_kernel(const double* __restrict__ x, int64_t n, Scratch s,
                                                       MArgs ma, int n_probs, int pass, int with_mean) {
    extern __shared__ uint32_t lds_hist[];   // [nq][kBins]
    __shared__ SelState cur[kMaxProbs];
    // pass 0 starts every probability from the empty prefix, so one histogram serves all
    const int nq = pass == 0 ? (n_probs > 0 ? 1 : 0) : n_probs;
    for (int i = threadIdx.x; i < nq * kBins; i += blockDim.x) lds_hist[i] = 0;
    for (int q = 0; q < n_probs; ++q) {
        // pass 0 starts from the empty prefix and records that state for pass 1
        SelState st{0, 0, ma.m[q], ma.m[q]};
        if (pass == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
            s.st[q] = st;
            s.ccount[q] = 0;
        }
        if (pass > 0) {
            st = s.st[((pass - 1) & 1) * kMaxProbs + q];
            // pass 0 fills the first probability's slot only: its histogram serves all
            st = choose_digit(s.hist + ((pass - 1) % 3) * kHistStride + int64_t(pass == 1 ? 0 : q) * kBins, st,
                              pass - 1);
            if (blockIdx.x == 0 && threadIdx.x == 0) s.st[(pass & 1) * kMaxProbs + q] = st;
        }
        if (threadIdx.x == 0) cur[q] = st;
    }
    {   // the histogram pass + 1 fills: last used two passes ago, so nobody touches it now
        uint32_t* nxt = s.hist + ((pass + 1) % 3) * kHistStride;
        const int64_t per = (int64_t(n_probs) * kBins + gridDim.x - 1) / gridDim.x;
        const int64_t b0 = per * blockIdx.x;
        for (int64_t i = b0 + threadIdx.x; i < b0 + per && i < int64_t(n_probs) * kBins; i += blockDim.x) nxt[i] = 0;
    }
    __syncthreads();
    const int shift = kShift[pass];
    const uint64_t dmask = (uint64_t(1) << kBits[pass]) - 1;
    uint64_t pre[kMaxProbs], msk[kMaxProbs];
    for (int q = 0; q < n_probs; ++q) {
        pre[q] = cur[q].prefix;
        msk[q] = cur[q].mask;
    }
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    uint32_t bad = 0;
    double mhi = 0.0, mlo = 0.0;
    auto take = [&](double v) {
        if (pass == 0 && !(v >= 0.0)) bad = 1;
        if (with_mean) dd_add(mhi, mlo, v);
        const uint64_t key = key_of(v);
        const uint32_t d = static_cast<uint32_t>((key >> shift) & dmask);
        for (int q = 0; q < nq; ++q)
            if ((key & msk[q]) == pre[q]) atomicAdd(&lds_hist[q * kBins + d], 1u);
    };
    // eight loads in flight per thread (all of a thread's values at the
    // launch's usual 2048 values per workgroup)
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += 8 * stride) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = i + u * stride < n ? x[i + u * stride] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i + u * stride < n) take(v[u]);
    }
    if (bad) atomicOr(s.flag, 1u);
    if (with_mean) {
        int64_t zero = 0;
        block_reduce_dd(mhi, mlo, zero);
        if (threadIdx.x == 0) {
            s.part_hi[blockIdx.x] = mhi;
            s.part_lo[blockIdx.x] = mlo;
            s.part_cnt[blockIdx.x] = 0;
        }
    }
    __syncthreads();
    uint32_t* h = s.hist + (pass % 3) * kHistStride;
    for (int k = threadIdx.x; k < nq * kBins; k += blockDim.x) {
        const uint32_t c = lds_hist[k];
        if (c) atomicAdd(&h[k], c);
    }
}

// After the two 12-bit passes: every workgroup chooses the second digit, so
// each probability has a 24-bit prefix that holds its m-th largest value
// (block 0 keeps the state in st[0]).  Values above the prefix's range are
// summed and counted into the tail partials (slot 1 + q); the keys inside it
// are appended to the probability's candidate list, one atomic per wave.
__global__ __launch_bounds__(256) void collect_kernel(const double* __restrict__ x, int64_t n, Scratch s,
                                                      int n_probs) {
    __shared__ uint64_t pre_s[kMaxProbs], msk_s[kMaxProbs];
    constexpr int done = 1;                         // the pass whose histogram is read
    for (int q = 0; q < n_probs; ++q) {
        SelState st = s.st[(done & 1) * kMaxProbs + q];
        st = choose_digit(s.hist + (done % 3) * kHistStride + int64_t(q) * kBins, st, done);
        if (threadIdx.x == 0) {
            pre_s[q] = st.prefix;
            msk_s[q] = st.mask;
            if (blockIdx.x == 0) s.st[((done + 1) & 1) * kMaxProbs + q] = st;
        }
    }
    __syncthreads();
    {   // the first pass's histogram, read for the last time by the second
        // pass, is cleared for the next call (with the error flag, cleared
        // by the last kernel, the scratch is then ready without an init)
        const int64_t per = (kHistStride + gridDim.x - 1) / gridDim.x;
        const int64_t b0 = per * blockIdx.x;
        for (int64_t i = b0 + threadIdx.x; i < b0 + per && i < kHistStride; i += blockDim.x) s.hist[i] = 0;
    }
    const int lane = threadIdx.x & 63;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    uint64_t pre[kMaxProbs], msk[kMaxProbs];
    double hi[kMaxProbs], lo[kMaxProbs];
    int64_t cnt[kMaxProbs];
#pragma unroll
    for (int q = 0; q < kMaxProbs; ++q) {
        pre[q] = q < n_probs ? pre_s[q] : 0;
        msk[q] = q < n_probs ? msk_s[q] : 0;
        hi[q] = 0.0;
        lo[q] = 0.0;
        cnt[q] = 0;
    }
    // each value is loaded once for every probability, eight loads in
    // flight per thread; whole waves step together (the bound is per
    // workgroup), so every lane takes part in the ballots
    for (int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x; b < n; b += 8 * stride) {
        double v[8];
        bool ok[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t i = b + u * stride + threadIdx.x;
            ok[u] = i < n;
            v[u] = ok[u] ? x[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint64_t key = key_of(v[u]);
#pragma unroll
            for (int q = 0; q < kMaxProbs; ++q) {
                if (q >= n_probs) break;
                const uint64_t top = pre[q] | ~msk[q];      // the largest key with the prefix
                if (ok[u] && key > top) {
                    dd_add(hi[q], lo[q], v[u]);
                    cnt[q] += 1;
                }
                const bool in = ok[u] && (key & msk[q]) == pre[q];
                const uint64_t bal = __ballot(in);
                if (bal) {
                    const int leader = __builtin_ctzll(bal);
                    uint32_t at = 0;
                    if (lane == leader) at = atomicAdd(&s.ccount[q], static_cast<uint32_t>(__popcll(bal)));
                    at = static_cast<uint32_t>(__shfl(static_cast<int>(at), leader, kWave));
                    if (in) s.cand[static_cast<int64_t>(q) * n + at + __popcll(bal & ((uint64_t(1) << lane) - 1))] = key;
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < kMaxProbs; ++q) {
        if (q >= n_probs) break;
        block_reduce_dd(hi[q], lo[q], cnt[q]);
        if (threadIdx.x == 0) {
            s.part_hi[(1 + q) * kSumBlocks + blockIdx.x] = hi[q];
            s.part_lo[(1 + q) * kSumBlocks + blockIdx.x] = lo[q];
            s.part_cnt[(1 + q) * kSumBlocks + blockIdx.x] = cnt[q];
        }
        __syncthreads();
    }
}

// One workgroup: the mean from the pass-0 partials; per probability, the
// remaining digits chosen over its candidates (histograms in LDS), then PML
// and TVaR from the tail partials plus the candidates above the threshold
// (fixed reduction order).  Every load that depends on no other is issued
// first (partials, states, candidate counts), then the candidates of each
// probability with few of them go to LDS, so the work waits for two round
// trips to memory instead of one or more per step.
__global__ __launch_bounds__(256) void finish_kernel(Scratch s, int n_probs, int n_mean_part, int n_tail_part,
                                                     int64_t n, MetricsOut out) {
    __shared__ __attribute__((aligned(16))) uint32_t hist[kBins];
    __shared__ uint64_t keys[kMaxProbs][kDirect];
    __shared__ uint64_t found;
    constexpr int kPer = kSumBlocks / 256;                  // partials per thread
    const bool bad = *s.flag != 0;
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    double mh[kPer], ml[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int i = threadIdx.x + u * 256;
        mh[u] = i < n_mean_part ? s.part_hi[i] : 0.0;
        ml[u] = i < n_mean_part ? s.part_lo[i] : 0.0;
    }
    SelState sq[kMaxProbs];
    int64_t cq[kMaxProbs];
    double th[kMaxProbs][kPer], tl[kMaxProbs][kPer];
    int64_t tc[kMaxProbs][kPer];
#pragma unroll
    for (int q = 0; q < kMaxProbs; ++q) {
        if (q >= n_probs) break;
        sq[q] = s.st[q];                            // written by the collect pass (st[0])
        cq[q] = static_cast<int64_t>(s.ccount[q]);
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int i = threadIdx.x + u * 256;
            const bool in = i < n_tail_part;
            th[q][u] = in ? s.part_hi[(1 + q) * kSumBlocks + i] : 0.0;
            tl[q][u] = in ? s.part_lo[(1 + q) * kSumBlocks + i] : 0.0;
            tc[q][u] = in ? s.part_cnt[(1 + q) * kSumBlocks + i] : 0;
        }
    }
#pragma unroll
    for (int q = 0; q < kMaxProbs; ++q) {
        if (q >= n_probs) break;
        if (cq[q] <= kDirect) {
            const uint64_t* cand = s.cand + static_cast<int64_t>(q) * n;
            for (int64_t j = threadIdx.x; j < cq[q]; j += blockDim.x) keys[q][j] = cand[j];
        }
    }
    __syncthreads();
    {
        double hi = 0.0, lo = 0.0;
        int64_t cnt = 0;
#pragma unroll
        for (int u = 0; u < kPer; ++u)
            if (threadIdx.x + u * 256 < n_mean_part) dd_merge(hi, lo, mh[u], ml[u]);
        block_reduce_dd(hi, lo, cnt);
        if (threadIdx.x == 0) *out.mean = bad ? nan : (hi + lo) / static_cast<double>(n);
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < kMaxProbs; ++q) {
        if (q >= n_probs) break;
        SelState st = sq[q];
        const int64_t c = cq[q];
        const uint64_t* cand = s.cand + static_cast<int64_t>(q) * n;
        const uint64_t* kq = keys[q];
        if (c <= kDirect) {
            // few candidates: the k-th largest is the key with fewer than k
            // keys above it and at least k at or above it
            for (int64_t j = threadIdx.x; j < c; j += blockDim.x) {
                const uint64_t kj = kq[j];
                int64_t gt = 0, ge = 0;
                for (int64_t i = 0; i < c; ++i) {
                    gt += kq[i] > kj;
                    ge += kq[i] >= kj;
                }
                if (gt < st.k && st.k <= ge) found = kj;      // every such thread writes the same key
            }
            __syncthreads();
            st.prefix = found;
            st.mask = ~uint64_t(0);
            __syncthreads();
        }
        for (int pass = 2; pass < kPasses && c > kDirect; ++pass) {
            for (int i = threadIdx.x; i < kBins; i += blockDim.x) hist[i] = 0;
            __syncthreads();
            const int shift = kShift[pass];
            const uint64_t dmask = (uint64_t(1) << kBits[pass]) - 1;
            for (int64_t j = threadIdx.x; j < c; j += blockDim.x) {
                const uint64_t key = cand[j];
                if ((key & st.mask) == st.prefix) atomicAdd(&hist[(key >> shift) & dmask], 1u);
            }
            __syncthreads();
            st = choose_digit(hist, st, pass);
        }
        const uint64_t vk = st.prefix;              // all 64 bits chosen: the m-th largest key
        double hi = 0.0, lo = 0.0;
        int64_t cnt = 0;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            if (threadIdx.x + u * 256 < n_tail_part) {
                dd_merge(hi, lo, th[q][u], tl[q][u]);
                cnt += tc[q][u];
            }
        }
        for (int64_t j = threadIdx.x; j < c; j += blockDim.x) {
            const uint64_t key = c <= kDirect ? kq[j] : cand[j];
            if (key > vk) {
                dd_add(hi, lo, __longlong_as_double(static_cast<long long>(key)));
                cnt += 1;
            }
        }
        block_reduce_dd(hi, lo, cnt);
        if (threadIdx.x == 0) {
            const double v = __longlong_as_double(static_cast<long long>(vk));
            const double r = static_cast<double>(st.m - cnt);   // copies of v in the top m
            const double p = r * v;
            const double pe = fma(r, v, -p);                   // exact product p + pe
            dd_merge(hi, lo, p, pe);
            out.pml[q * out.stride] = bad ? nan : v;
            out.tvar[q * out.stride] = bad ? nan : (hi + lo) / static_cast<double>(st.m);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *s.flag = 0;              // read by every thread before the barriers above
}

// one workgroup: the mean from the pass-0 partials, then PML and TVaR per
// probability from the tail partials (fixed reduction order)
__global__ __launch_bounds__(256) void final_kernel(Scratch s, int n_probs, int n_mean_part, int n_tail_part,
                                                    int64_t n, MetricsOut out) {
    const bool bad = *s.flag != 0;
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    for (int slot = 0; slot <= n_probs; ++slot) {
        const int np = slot == 0 ? n_mean_part : n_tail_part;
        double hi = 0.0, lo = 0.0;
        int64_t cnt = 0;
        for (int i = threadIdx.x; i < np; i += blockDim.x) {
            dd_merge(hi, lo, s.part_hi[slot * kSumBlocks + i], s.part_lo[slot * kSumBlocks + i]);
            cnt += s.part_cnt[slot * kSumBlocks + i];
        }
        block_reduce_dd(hi, lo, cnt);
        if (threadIdx.x == 0) {
            if (slot == 0) {
                *out.mean = bad ? nan : (hi + lo) / static_cast<double>(n);
            } else {
                const int q = slot - 1;
                const SelState st = s.st[((kPasses) & 1) * kMaxProbs + q];
                const double v = __longlong_as_double(static_cast<long long>(st.prefix));
                const double r = static_cast<double>(st.m - cnt);   // copies of v in the top m
                const double p = r * v;
                const double pe = fma(r, v, -p);                   // exact product p + pe
                dd_merge(hi, lo, p, pe);
                out.pml[q * out.stride] = bad ? nan : v;
                out.tvar[q * out.stride] = bad ? nan : (hi + lo) / static_cast<double>(st.m);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *s.flag = 0;              // read by every thread before the barriers above
}

// one workgroup: the final digit for the single tail count, into `out`


}  // namespace

int64_t metrics_scratch_bytes(int n_probs, int64_t n) {
    const int64_t base = (base_bytes() + kCandAlign - 1) / kCandAlign * kCandAlign;
    return base + static_cast<int64_t>(n_probs) * n * static_cast<int64_t>(sizeof(uint64_t));
}

namespace {
// workgroups of `threads` threads for eight values per thread, at most kSumBlocks
int hist_blocks(int64_t n, int threads) {
    const int64_t per = static_cast<int64_t>(threads) * 8;
    int64_t b = (n + per - 1) / per;
    if (b > kSumBlocks) b = kSumBlocks;
    if (b < 1) b = 1;
    return static_cast<int>(b);
}
}  // namespace

hipError_t launch_metrics_prime(void* scratch, const int64_t* m_host, int n_probs, hipStream_t st) {
    if (n_probs > kMaxProbs) return hipErrorInvalidValue;
    Scratch s = carve(scratch, n_probs);
    MArgs ma{};
    for (int q = 0; q < n_probs; ++q) ma.m[q] = m_host[q];
    hipLaunchKernelGGL(select_init_kernel, dim3(16), dim3(256), 0, st, s, ma, n_probs);
    return hipGetLastError();
}

hipError_t launch_metrics(const double* ylt, int64_t n, const int64_t* m_host, int n_probs,
                          void* scratch, bool primed, MetricsOut out, int n_cu, hipStream_t st) {
    if (n_probs > kMaxProbs) return hipErrorInvalidValue;
    (void)n_cu;
    Scratch s = carve(scratch, n_probs);
    MArgs ma{};
    for (int q = 0; q < n_probs; ++q) ma.m[q] = m_host[q];
    hipError_t err;
    // a scratch left by a completed call has a clear first histogram and a
    // clear error flag; only a new one (or one after a failed launch) needs this
    if (!primed) {
        hipLaunchKernelGGL(select_init_kernel, dim3(16), dim3(256), 0, st, s, ma, n_probs);
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    // two 12-bit passes (the first also sums for the mean), then one pass that
    // sums the tail above each 24-bit prefix and collects the keys inside it,
    // and one workgroup that finishes the selection over those candidates
    const int h0 = hist_blocks(n, kHist0Threads), h1 = hist_blocks(n, kHist1Threads);
    hipLaunchKernelGGL(histogram_kernel<kHist0Threads>, dim3(h0), dim3(kHist0Threads), sizeof(uint32_t) * kBins, st,
                       ylt, n, s, ma, n_probs, 0, 1);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if (n_probs == 0) {
        hipLaunchKernelGGL(final_kernel, dim3(1), dim3(256), 0, st, s, 0, h0, 1, n, out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(histogram_kernel<kHist1Threads>, dim3(h1), dim3(kHist1Threads),
                       sizeof(uint32_t) * kBins * n_probs, st, ylt, n, s, ma, n_probs, 1, 0);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    int tblocks = static_cast<int>((n + 1023) / 1024);
    if (tblocks > kSumBlocks) tblocks = kSumBlocks;
    if (tblocks < 1) tblocks = 1;
    hipLaunchKernelGGL(collect_kernel, dim3(tblocks), dim3(256), 0, st, ylt, n, s, n_probs);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(256), 0, st, s, n_probs, h0, tblocks, n, out);
    return hipGetLastError();
}

}  // namespace ara

namespace ara {

int64_t tail_stats_scratch_bytes(int64_t n) { return metrics_scratch_bytes(1, n); }

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept; later calls reuse it.  No
// allocation of any kind.
hipError_t metrics_noalloc_scratch(void** ptr, int64_t* capacity) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *capacity = kStaticBytes;
    return hipSuccess;
}

namespace {

// After collect_kernel for one tail count m: the m-th largest key, chosen
// among the candidates inside its 24-bit prefix as finish_kernel does, the
// count of year losses above it (those above the prefix, counted by
// collect_kernel, plus the candidates above it) and the count equal to it
// (all of them are candidates).  One workgroup.
__global__ __launch_bounds__(256) void tail_select_kernel(Scratch s, int n_tail_part, TailStats* out) {
    __shared__ __attribute__((aligned(16))) uint32_t hist[kBins];
    __shared__ uint64_t keys[kDirect];
    __shared__ uint64_t found;
    __shared__ unsigned long long red[2][4];
    SelState st = s.st[0];                          // written by the collect pass
    const int64_t c = static_cast<int64_t>(s.ccount[0]);
    const uint64_t* cand = s.cand;
    if (c <= kDirect) {
        for (int64_t j = threadIdx.x; j < c; j += blockDim.x) keys[j] = cand[j];
        __syncthreads();
        for (int64_t j = threadIdx.x; j < c; j += blockDim.x) {
            const uint64_t kj = keys[j];
            int64_t gt = 0, ge = 0;
            for (int64_t i = 0; i < c; ++i) {
                gt += keys[i] > kj;
                ge += keys[i] >= kj;
            }
            if (gt < st.k && st.k <= ge) found = kj;          // every such thread writes the same key
        }
        __syncthreads();
        st.prefix = found;
        st.mask = ~uint64_t(0);
        __syncthreads();
    }
    for (int pass = 2; pass < kPasses && c > kDirect; ++pass) {
        for (int i = threadIdx.x; i < kBins; i += blockDim.x) hist[i] = 0;
        __syncthreads();
        const int shift = kShift[pass];
        const uint64_t dmask = (uint64_t(1) << kBits[pass]) - 1;
        for (int64_t j = threadIdx.x; j < c; j += blockDim.x) {
            const uint64_t key = cand[j];
            if ((key & st.mask) == st.prefix) atomicAdd(&hist[(key >> shift) & dmask], 1u);
        }
        __syncthreads();
        st = choose_digit(hist, st, pass);
    }
    const uint64_t vk = st.prefix;
    unsigned long long gt = 0, eq = 0;
    for (int i = threadIdx.x; i < n_tail_part; i += blockDim.x)
        gt += static_cast<unsigned long long>(s.part_cnt[kSumBlocks + i]);
    for (int64_t j = threadIdx.x; j < c; j += blockDim.x) {
        const uint64_t key = cand[j];
        gt += key > vk;
        eq += key == vk;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        gt += __shfl_xor(gt, off, kWave);
        eq += __shfl_xor(eq, off, kWave);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = gt;
        red[1][threadIdx.x >> 6] = eq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out->v_bits = vk;
        out->m = st.m;
        out->c_gt = static_cast<int64_t>(red[0][0] + red[0][1] + red[0][2] + red[0][3]);
        out->c_eq = static_cast<int64_t>(red[1][0] + red[1][1] + red[1][2] + red[1][3]);
    }
}

}  // namespace

// the m-th largest year loss with the counts above and at it: the selection of
// launch_metrics (two 12-bit passes, the candidates inside the 24-bit prefix,
// one workgroup over them), five launches
hipError_t launch_tail_stats(const double* ylt, int64_t n, int64_t m, void* scratch, TailStats* out,
                             int n_cu, hipStream_t st) {
    (void)n_cu;
    Scratch s = carve(scratch, 1);
    MArgs ma{};
    ma.m[0] = m;
    hipError_t err;
    hipLaunchKernelGGL(select_init_kernel, dim3(16), dim3(256), 0, st, s, ma, 1);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(histogram_kernel<kHist0Threads>, dim3(hist_blocks(n, kHist0Threads)), dim3(kHist0Threads),
                       sizeof(uint32_t) * kBins, st, ylt, n, s, ma, 1, 0, 0);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(histogram_kernel<kHist1Threads>, dim3(hist_blocks(n, kHist1Threads)), dim3(kHist1Threads),
                       sizeof(uint32_t) * kBins, st, ylt, n, s, ma, 1, 1, 0);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    int tblocks = static_cast<int>((n + 1023) / 1024);
    if (tblocks > kSumBlocks) tblocks = kSumBlocks;
    if (tblocks < 1) tblocks = 1;
    hipLaunchKernelGGL(collect_kernel, dim3(tblocks), dim3(256), 0, st, ylt, n, s, 1);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(tail_select_kernel, dim3(1), dim3(256), 0, st, s, tblocks, out);
    return hipGetLastError();
}

}  // namespace ara
