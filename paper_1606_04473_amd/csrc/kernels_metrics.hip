// Risk metrics from a Year Loss Table: mean, PML_p, TVaR_p.
//
// Year losses are >= 0, so their IEEE-754 bit patterns order like their
// values when read as uint64.  PML_p (the m-th largest) is found by a radix
// select over those patterns: six passes with 12/12/12/12/12/4-bit digits,
// each pass a privatised LDS histogram of the values that match the prefix
// chosen so far, followed by a one-workgroup digit choice.  All requested
// probabilities advance together in each pass.  TVaR_p = (sum of the values
// above v + (m - c_gt) v) / m, with v = PML_p and c_gt the count above it.
// Sums are double-double, reduced in a fixed order (deterministic), and the
// product (m - c_gt) v is added exactly via fma.
#include "ara_internal.hpp"

namespace ara {

namespace {

constexpr int kSumBlocks = 512;
constexpr int kBins = 4096;
constexpr int kPasses = 6;
constexpr int kMaxProbs = 4;   // 4 x 16 KB histograms fit the 64 KB dynamic-LDS default
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
    uint32_t* hist;       // [n_probs][kBins]
    SelState* st;         // [n_probs]
    uint32_t* flag;
};

Scratch carve(void* base, int n_probs) {
    char* p = static_cast<char*>(base);
    Scratch s;
    const int64_t np = static_cast<int64_t>(kMaxProbs + 1) * kSumBlocks;
    s.part_hi = reinterpret_cast<double*>(p);
    p += np * sizeof(double);
    s.part_lo = reinterpret_cast<double*>(p);
    p += np * sizeof(double);
    s.part_cnt = reinterpret_cast<int64_t*>(p);
    p += np * sizeof(int64_t);
    s.hist = reinterpret_cast<uint32_t*>(p);
    p += static_cast<int64_t>(n_probs) * kBins * sizeof(uint32_t);
    s.st = reinterpret_cast<SelState*>(p);
    p += static_cast<int64_t>(kMaxProbs) * sizeof(SelState);
    s.flag = reinterpret_cast<uint32_t*>(p);
    return s;
}

__device__ __forceinline__ uint64_t key_of(double x) {
    // +0.0 for -0.0 so that zero losses of either sign rank lowest
    return __double_as_longlong(x + 0.0);
}

// block-wide double-double reduction; result valid in thread 0
__device__ __forceinline__ void block_reduce_dd(double& hi, double& lo, int64_t& cnt) {
    __shared__ double sh[4], sl[4];
    __shared__ int64_t sc[4];
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

// mode 0: sum of all values (slot 0); mode 1: for each prob q, sum and
// count of the values strictly above its selected threshold (slot 1 + q)
template <int MODE>
__global__ __launch_bounds__(256) void partial_sums_kernel(const double* __restrict__ x, int64_t n,
                                                           Scratch s, int n_probs) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int nq = MODE == 0 ? 1 : n_probs;
    for (int q = 0; q < nq; ++q) {
        double hi = 0.0, lo = 0.0;
        int64_t cnt = 0;
        const uint64_t thr = MODE == 0 ? 0 : s.st[q].prefix;
        for (int64_t i = tid; i < n; i += stride) {
            const double v = x[i];
            if (MODE == 0) {
                dd_add(hi, lo, v);
            } else if (key_of(v) > thr) {
                dd_add(hi, lo, v);
                cnt += 1;
            }
        }
        block_reduce_dd(hi, lo, cnt);
        if (threadIdx.x == 0) {
            const int slot = MODE == 0 ? 0 : 1 + q;
            s.part_hi[slot * kSumBlocks + blockIdx.x] = hi;
            s.part_lo[slot * kSumBlocks + blockIdx.x] = lo;
            s.part_cnt[slot * kSumBlocks + blockIdx.x] = cnt;
        }
        __syncthreads();
    }
}

template <int MODE>
__global__ __launch_bounds__(64) void final_sums_kernel(Scratch s, int n_probs, int n_part, int64_t n,
                                                        MetricsOut out) {
    const int nq = MODE == 0 ? 1 : n_probs;
    const bool bad = *s.flag != 0;
    for (int q = 0; q < nq; ++q) {
        const int slot = MODE == 0 ? 0 : 1 + q;
        double hi = 0.0, lo = 0.0;
        int64_t cnt = 0;
        for (int i = threadIdx.x; i < n_part; i += kWave) {
            dd_merge(hi, lo, s.part_hi[slot * kSumBlocks + i], s.part_lo[slot * kSumBlocks + i]);
            cnt += s.part_cnt[slot * kSumBlocks + i];
        }
        group_reduce_dd(hi, lo, kWave);
        for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, kWave);
        if (threadIdx.x == 0) {
            const double nan = __longlong_as_double(0x7ff8000000000000LL);
            if (MODE == 0) {
                *out.mean = bad ? nan : (hi + lo) / static_cast<double>(n);
            } else {
                const SelState st = s.st[q];
                const double v = __longlong_as_double(static_cast<long long>(st.prefix));
                const double r = static_cast<double>(st.m - cnt);   // copies of v in the top m
                const double p = r * v;
                const double pe = fma(r, v, -p);                   // exact product p + pe
                dd_merge(hi, lo, p, pe);
                out.pml[q * out.stride] = bad ? nan : v;
                out.tvar[q * out.stride] = bad ? nan : (hi + lo) / static_cast<double>(st.m);
            }
        }
    }
}

struct MArgs {
    int64_t m[kMaxProbs];
};

// resets the selection state and clears the histograms with plain stores
__global__ void select_init_kernel(Scratch s, MArgs ma, int n_probs) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < n_probs) {
        s.st[tid].prefix = 0;
        s.st[tid].mask = 0;
        s.st[tid].k = ma.m[tid];
        s.st[tid].m = ma.m[tid];
    }
    if (tid == 0) *s.flag = 0;
    for (int i = tid; i < n_probs * kBins; i += gridDim.x * blockDim.x) s.hist[i] = 0;
}

__global__ __launch_bounds__(256) void histogram_kernel(const double* __restrict__ x, int64_t n, Scratch s,
                                                        int n_probs, int pass, int with_mean) {
    extern __shared__ uint32_t lds_hist[];   // [n_probs][kBins]
    for (int i = threadIdx.x; i < n_probs * kBins; i += blockDim.x) lds_hist[i] = 0;
    __syncthreads();
    const int shift = kShift[pass];
    const uint64_t dmask = (uint64_t(1) << kBits[pass]) - 1;
    uint64_t pre[kMaxProbs], msk[kMaxProbs];
    for (int q = 0; q < n_probs; ++q) {
        pre[q] = s.st[q].prefix;
        msk[q] = s.st[q].mask;
    }
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    uint32_t bad = 0;
    double mhi = 0.0, mlo = 0.0;
    auto take = [&](double v) {
        if (pass == 0 && !(v >= 0.0)) bad = 1;
        if (with_mean) dd_add(mhi, mlo, v);
        const uint64_t key = key_of(v);
        const uint32_t d = static_cast<uint32_t>((key >> shift) & dmask);
        for (int q = 0; q < n_probs; ++q)
            if ((key & msk[q]) == pre[q]) atomicAdd(&lds_hist[q * kBins + d], 1u);
    };
    // four loads in flight per thread, then the tail
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const double v0 = x[i], v1 = x[i + stride], v2 = x[i + 2 * stride], v3 = x[i + 3 * stride];
        take(v0);
        take(v1);
        take(v2);
        take(v3);
    }
    for (; i < n; i += stride) take(x[i]);
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
    for (int i = threadIdx.x; i < n_probs * kBins; i += blockDim.x) {
        const uint32_t c = lds_hist[i];
        if (c) atomicAdd(&s.hist[i], c);
    }
}

// one workgroup of 256 threads per probability: choose the digit holding the
// k-th largest remaining value, then clear the histogram for the next pass
__global__ __launch_bounds__(256) void select_digit_kernel(Scratch s, int pass) {
    const int q = blockIdx.x;
    uint32_t* h = s.hist + static_cast<int64_t>(q) * kBins;
    const int nb = 1 << kBits[pass];
    const int per = (nb + 255) / 256;
    // thread i owns bins [nb - per (i+1), nb - per i): thread 0 the largest digits
    const int hiBin = nb - per * threadIdx.x;
    const int loBin = hiBin - per;
    uint64_t local = 0;
    for (int b = hiBin - 1; b >= loBin && b >= 0; --b) local += h[b];
    __shared__ uint64_t scan[256];
    scan[threadIdx.x] = local;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint64_t add = threadIdx.x >= off ? scan[threadIdx.x - off] : 0;
        __syncthreads();
        scan[threadIdx.x] += add;
        __syncthreads();
    }
    const uint64_t incl = scan[threadIdx.x];
    const uint64_t excl = incl - local;
    const SelState st = s.st[q];
    const uint64_t k = static_cast<uint64_t>(st.k);
    __syncthreads();
    if (excl < k && k <= incl) {
        uint64_t cum = excl;
        for (int b = hiBin - 1; b >= loBin && b >= 0; --b) {
            const uint64_t c = h[b];
            if (cum + c >= k) {
                const int shift = kShift[pass];
                const uint64_t dmask = (uint64_t(1) << kBits[pass]) - 1;
                s.st[q].k = static_cast<int64_t>(k - cum);
                s.st[q].prefix = st.prefix | (static_cast<uint64_t>(b) << shift);
                s.st[q].mask = st.mask | (dmask << shift);
                break;
            }
            cum += c;
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kBins; b += 256) h[b] = 0;
}

__global__ void tail_finish_kernel(Scratch s, TailStats* out) {
    if (threadIdx.x == 0) {
        out->v_bits = s.st[0].prefix;
        out->m = s.st[0].m;
        out->c_gt = 0;
        out->c_eq = 0;
    }
}

__global__ __launch_bounds__(256) void tail_count_kernel(const double* __restrict__ x, int64_t n,
                                                         TailStats* out) {
    const uint64_t v = out->v_bits;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    unsigned long long gt = 0, eq = 0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t k = key_of(x[i]);
        gt += k > v;
        eq += k == v;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        gt += __shfl_xor(gt, off, kWave);
        eq += __shfl_xor(eq, off, kWave);
    }
    if ((threadIdx.x & 63) == 0) {
        if (gt) atomicAdd(reinterpret_cast<unsigned long long*>(&out->c_gt), gt);
        if (eq) atomicAdd(reinterpret_cast<unsigned long long*>(&out->c_eq), eq);
    }
}

}  // namespace

int64_t metrics_scratch_bytes(int n_probs) {
    const int64_t np = static_cast<int64_t>(kMaxProbs + 1) * kSumBlocks;
    return np * (2 * sizeof(double) + sizeof(int64_t)) +
           static_cast<int64_t>(n_probs) * kBins * sizeof(uint32_t) + kMaxProbs * sizeof(SelState) +
           64;
}

hipError_t launch_metrics(const double* ylt, int64_t n, const int64_t* m_host, int n_probs,
                          void* scratch, MetricsOut out, int n_cu, hipStream_t st) {
    if (n_probs > kMaxProbs) return hipErrorInvalidValue;
    Scratch s = carve(scratch, n_probs);
    MArgs ma{};
    for (int q = 0; q < n_probs; ++q) ma.m[q] = m_host[q];
    hipError_t err;
    hipLaunchKernelGGL(select_init_kernel, dim3(16), dim3(256), 0, st, s, ma, n_probs);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    // enough workgroups to keep many loads in flight; each adds only its
    // non-zero bins to the global histogram (values crowd into few bins)
    int hblocks = static_cast<int>((n + 2047) / 2048);
    if (hblocks > kSumBlocks) hblocks = kSumBlocks;
    if (hblocks < 1) hblocks = 1;
    (void)n_cu;
    const size_t lds = sizeof(uint32_t) * kBins * (n_probs > 0 ? n_probs : 1);
    const int passes = n_probs > 0 ? kPasses : 1;
    for (int pass = 0; pass < passes; ++pass) {
        hipLaunchKernelGGL(histogram_kernel, dim3(hblocks), dim3(256), lds, st, ylt, n, s, n_probs, pass,
                           pass == 0 ? 1 : 0);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        if (n_probs > 0) {
            hipLaunchKernelGGL(select_digit_kernel, dim3(n_probs), dim3(256), 0, st, s, pass);
            if ((err = hipGetLastError()) != hipSuccess) return err;
        }
    }
    hipLaunchKernelGGL((final_sums_kernel<0>), dim3(1), dim3(64), 0, st, s, n_probs, hblocks, n, out);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if (n_probs > 0) {
        int blocks = static_cast<int>((n + 1023) / 1024);
        if (blocks > kSumBlocks) blocks = kSumBlocks;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL((partial_sums_kernel<1>), dim3(blocks), dim3(256), 0, st, ylt, n, s, n_probs);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        hipLaunchKernelGGL((final_sums_kernel<1>), dim3(1), dim3(64), 0, st, s, n_probs, blocks, n, out);
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    return hipSuccess;
}

}  // namespace ara

namespace ara {

int64_t tail_stats_scratch_bytes() { return metrics_scratch_bytes(1); }

hipError_t launch_tail_stats(const double* ylt, int64_t n, int64_t m, void* scratch, TailStats* out,
                             int n_cu, hipStream_t st) {
    Scratch s = carve(scratch, 1);
    MArgs ma{};
    ma.m[0] = m;
    hipError_t err;
    hipLaunchKernelGGL(select_init_kernel, dim3(16), dim3(256), 0, st, s, ma, 1);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    int hblocks = static_cast<int>((n + 1023) / 1024);
    if (hblocks > 2 * n_cu) hblocks = 2 * n_cu;
    if (hblocks < 1) hblocks = 1;
    for (int pass = 0; pass < kPasses; ++pass) {
        hipLaunchKernelGGL(histogram_kernel, dim3(hblocks), dim3(256), sizeof(uint32_t) * kBins, st, ylt, n, s,
                           1, pass, 0);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        hipLaunchKernelGGL(select_digit_kernel, dim3(1), dim3(256), 0, st, s, pass);
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    hipLaunchKernelGGL(tail_finish_kernel, dim3(1), dim3(64), 0, st, s, out);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(tail_count_kernel, dim3(hblocks), dim3(256), 0, st, ylt, n, out);
    return hipGetLastError();
}

}  // namespace ara
