// Adjoint of the year loss with respect to a layer's terms.
//
// With the strict convention at kinks every partial of YLT_t is an integer:
//   d YLT_t / d theta_k = a_t * sum over the trial's occurrences of g_k(E)
// for the per-ELT and occurrence terms, where a_t = [0 < S_t - AggR < AggL]
// and g_k(E) in {-1, 0, 1} depends on the event only; dYLT_t/dAggR = -a_t and
// dYLT_t/dAggL = [S_t - AggR > AggL].  Summing over trials with weights w_t
// (1 for the mean; for TVaR c_eq above the m-th largest value v and m - c_gt
// at v) regroups by event:
//   sum_t w_t a_t sum_d g_k(E_td) = sum_E g_k(E) * W(E),
//   W(E) = sum over active trials of w_t * (multiplicity of E in trial t).
// So the backward is one pass over the events of active trials that builds
// the integer histogram W (only for events whose occurrence loss can move:
// y(E) - OccR > 0), then one pass over the catalogue that evaluates g(E)
// with the forward's FP64 operations and accumulates g_k(E) W(E) in int64.
// Integer atomics make the result independent of scheduling.
#include "ara_internal.hpp"

namespace ara {

namespace {

constexpr int kMaxP = 2 * kMaxJ + 4;

// signed 64-bit add through the unsigned atomic (two's complement wraps)
__device__ __forceinline__ void add_i64(long long* p, long long v) {
    atomicAdd(reinterpret_cast<unsigned long long*>(p), static_cast<unsigned long long>(v));
}

struct AdjScratch {
    uint8_t* mark;         // [C]
    uint64_t* w_mean;      // [C]
    uint64_t* w_tvar;      // [C]
    long long* acc;        // [2][kMaxP] integer numerators
    TailStats* tail;
    void* cls;             // trial classes of the stream histogram
    int64_t cls_bytes;
    void* tail_scratch;
};

// The same numerators from the sparse ELT pool: one workgroup per chunk of
// kSparseChunk events.  y(E) is rebuilt in LDS as the forward fold does it
// (each ELT's entries added in layer order; an absent loss would add +0.0),
// so it is bit-identical to the dense sum.  Each event with a weight then adds
// its occurrence-term slopes, and each nonzero loss (E, l) of ELT j its
// per-ELT slopes; an absent loss has l - R_j <= 0 and no slope, so the sparse
// entries give the dense kernel's integer sums.
//
// The chunk's entries of the layer's ELTs (in layer order) are first copied to
// LDS, kStage at a time, with all their loads in flight together; the fold
// and the per-ELT slopes then read LDS only, so the ordered fold costs one
// barrier per ELT and no memory latency.  The weights of the chunk's events
// are kept in LDS for the slopes.
constexpr int kSparseChunk = 4096;                  // events per chunk of the sparse pool
constexpr int kStage = 4096;                        // pool entries staged in LDS at a time

// sum over the wave's lanes
__device__ __forceinline__ long long wave_sum_i64(long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__global__ __launch_bounds__(1024) void catalogue_sparse_kernel(SparsePool sp, int64_t C, LayerArgs L,
                                                                const uint64_t* __restrict__ w_mean,
                                                                const uint64_t* __restrict__ w_tvar,
                                                                long long* __restrict__ acc) {
    __shared__ double ys[kSparseChunk];
    __shared__ long long wms[kSparseChunk], wvs[kSparseChunk];
    __shared__ uint8_t act[kSparseChunk];           // inside the occurrence band, with a weight
    __shared__ double s_val[kStage];
    __shared__ uint16_t s_ev[kStage];
    __shared__ uint8_t s_j[kStage];
    __shared__ long long lacc[2 * kMaxP];
    __shared__ int64_t rb[kMaxJ], pre[kMaxJ + 1];
    __shared__ double sR[kMaxJ], sLim[kMaxJ];
    const int t = threadIdx.x;
    const int nt = blockDim.x;
    const int64_t chunk = blockIdx.x;
    const int64_t e0 = chunk * kSparseChunk;
    const int J = L.J;
    const int P = 2 * J + 4;
    for (int i = t; i < kSparseChunk; i += nt) ys[i] = 0.0;
    for (int i = t; i < 2 * kMaxP; i += nt) lacc[i] = 0;
    if (t < J) {
        sR[t] = L.R[t];
        sLim[t] = L.Lim[t];
    }
    if (t == 0) {
        int64_t run = 0;
        for (int j = 0; j < J; ++j) {
            const int64_t key = static_cast<int64_t>(L.idx[j]) * sp.n_chunks + chunk;
            const int64_t b = sp.chunk_off[key];
            rb[j] = b;
            pre[j] = run;
            run += sp.chunk_off[key + 1] - b;
        }
        pre[J] = run;
    }
    __syncthreads();
    const int64_t n_ent = pre[J];
    // entries [r0, r0 + nr) of the chunk's list (ELT by ELT) to LDS
    auto stage = [&](int64_t r0, int nr) {
        for (int i = t; i < nr; i += nt) {
            const int64_t f = r0 + i;
            int lo = 0, hi = J;                     // the ELT whose range holds f: pre[lo] <= f < pre[lo + 1]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (pre[mid] <= f) lo = mid; else hi = mid;
            }
            const int64_t k = rb[lo] + (f - pre[lo]);
            s_ev[i] = sp.ev[k];
            s_val[i] = sp.val[k];
            s_j[i] = static_cast<uint8_t>(lo);
        }
    };
    // the fold, ELT by ELT in layer order
    for (int64_t r0 = 0; r0 < n_ent; r0 += kStage) {
        const int nr = static_cast<int>(n_ent - r0 < kStage ? n_ent - r0 : kStage);
        __syncthreads();                            // the previous round's entries are used
        stage(r0, nr);
        __syncthreads();
        for (int j = 0; j < J; ++j) {
            const int64_t a = pre[j] > r0 ? pre[j] : r0;
            const int64_t b = pre[j + 1] < r0 + nr ? pre[j + 1] : r0 + nr;
            if (a >= b) continue;                   // uniform: no ELT j entries in this round
            const double R = L.R[j], Lim = L.Lim[j];
            for (int64_t f = a + t; f < b; f += nt) {
                const int i = static_cast<int>(f - r0);
                const int ev = s_ev[i];
                ys[ev] = ys[ev] + apply_terms(s_val[i], R, Lim);
            }
            __syncthreads();
        }
    }
    // occurrence-term slopes; the events' weights and band flags to LDS
    {
        long long over_m = 0, over_v = 0, in_m = 0, in_v = 0;
        for (int i = t; i < kSparseChunk; i += nt) {
            const int64_t e = e0 + i;
            long long wm = 0, wv = 0;
            uint8_t a = 0;
            if (e < C) {
                wm = static_cast<long long>(w_mean[e]);
                wv = static_cast<long long>(w_tvar[e]);
                if (wm != 0 || wv != 0) {
                    const double to = ys[i] - L.occR;
                    if (to > L.occL) {
                        over_m += wm;
                        over_v += wv;
                    }
                    if ((to > 0.0) && (to < L.occL)) {
                        in_m += wm;
                        in_v += wv;
                        a = 1;
                    }
                }
            }
            wms[i] = wm;
            wvs[i] = wv;
            act[i] = a;
        }
        over_m = wave_sum_i64(over_m);
        over_v = wave_sum_i64(over_v);
        in_m = wave_sum_i64(in_m);
        in_v = wave_sum_i64(in_v);
        if ((t & 63) == 0) {
            if (over_m) add_i64(&lacc[2 * J + 1], over_m);
            if (over_v) add_i64(&lacc[kMaxP + 2 * J + 1], over_v);
            if (in_m) add_i64(&lacc[2 * J], -in_m);
            if (in_v) add_i64(&lacc[kMaxP + 2 * J], -in_v);
        }
    }
    // per-ELT slopes of the events inside the occurrence band (the staged
    // entries are still in LDS when the list fit in one round)
    for (int64_t r0 = 0; r0 < n_ent; r0 += kStage) {
        const int nr = static_cast<int>(n_ent - r0 < kStage ? n_ent - r0 : kStage);
        __syncthreads();
        if (n_ent > kStage) {
            stage(r0, nr);
            __syncthreads();
        }
        for (int i = t; i < nr; i += nt) {
            const int ev = s_ev[i];
            if (!act[ev]) continue;
            const int j = s_j[i];
            const long long wm = wms[ev], wv = wvs[ev];
            const double tj = s_val[i] - sR[j];
            const double Lim = sLim[j];
            if (tj > 0.0 && tj < Lim) {
                add_i64(&lacc[j], -wm);
                if (wv) add_i64(&lacc[kMaxP + j], -wv);
            }
            if (tj > Lim) {
                add_i64(&lacc[J + j], wm);
                if (wv) add_i64(&lacc[kMaxP + J + j], wv);
            }
        }
    }
    __syncthreads();
    for (int i = t; i < 2 * kMaxP; i += nt) {
        const int q = i % kMaxP;
        if (q < P - 2 && lacc[i] != 0) add_i64(&acc[i], lacc[i]);
    }
}

__global__ __launch_bounds__(256) void mark_kernel(const double* __restrict__ elts, int64_t C, LayerArgs L,
                                                   uint8_t* __restrict__ mark, uint64_t* __restrict__ w_mean,
                                                   uint64_t* __restrict__ w_tvar, int with_mark) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= C) return;
    w_mean[e] = 0;
    w_tvar[e] = 0;
    if (!with_mark) return;
    double y = 0.0;
    for (int j = 0; j < L.J; ++j)
        y = y + apply_terms(elts[static_cast<int64_t>(L.idx[j]) * C + e], L.R[j], L.Lim[j]);
    mark[e] = (y - L.occR > 0.0) ? 1 : 0;
}

__global__ void clear_acc_kernel(long long* acc) {
    for (int i = threadIdx.x; i < 2 * kMaxP; i += blockDim.x) acc[i] = 0;
}

// one wavefront per trial; only trials inside the aggregate band read events
__global__ __launch_bounds__(256) void active_trials_kernel(const int64_t* __restrict__ offsets,
                                                            const uint32_t* __restrict__ ids, LayerArgs L,
                                                            const double* __restrict__ S,
                                                            const double* __restrict__ ylt,
                                                            const TailStats* __restrict__ tail,
                                                            const uint8_t* __restrict__ mark,
                                                            uint64_t* __restrict__ w_mean,
                                                            uint64_t* __restrict__ w_tvar,
                                                            long long* __restrict__ acc) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = uniform_i64((static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6);
    const int64_t n_waves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
    const TailStats ts = *tail;
    const int P = 2 * L.J + 4;
    long long agg_r_mean = 0, agg_l_mean = 0, agg_r_tvar = 0, agg_l_tvar = 0;
    for (int64_t k = wave; k < L.trial_count; k += n_waves) {
        const double ta = S[k] - L.aggR;
        const bool in_band = (ta > 0.0) && (ta < L.aggL);
        const bool above = ta > L.aggL;
        const uint64_t key = __double_as_longlong(ylt[k] + 0.0);
        const long long wt = key > ts.v_bits ? ts.c_eq : (key == ts.v_bits ? ts.m - ts.c_gt : 0);
        if (in_band) {
            agg_r_mean -= 1;
            agg_r_tvar -= wt;
        }
        if (above) {
            agg_l_mean += 1;
            agg_l_tvar += wt;
        }
        if (!in_band) continue;
        const int64_t t = L.trial_begin + k;
        const int64_t b = offsets[t];
        const int64_t e = offsets[t + 1];
        for (int64_t i = b + lane; i < e; i += kWave) {
            const uint32_t id = ids[i];
            if (mark[id]) {
                atomicAdd(reinterpret_cast<unsigned long long*>(&w_mean[id]), 1ull);
                if (wt) atomicAdd(reinterpret_cast<unsigned long long*>(&w_tvar[id]),
                                  static_cast<unsigned long long>(wt));
            }
        }
    }
    if (lane == 0) {
        if (agg_r_mean) add_i64(&acc[P - 2], agg_r_mean);
        if (agg_l_mean) add_i64(&acc[P - 1], agg_l_mean);
        if (agg_r_tvar) add_i64(&acc[kMaxP + P - 2], agg_r_tvar);
        if (agg_l_tvar) add_i64(&acc[kMaxP + P - 1], agg_l_tvar);
    }
}

// aggregate-term partials alone (the partitioned histogram pass leaves them out)
__global__ __launch_bounds__(256) void agg_counts_kernel(LayerArgs L, const double* __restrict__ S,
                                                         const double* __restrict__ ylt,
                                                         const TailStats* __restrict__ tail,
                                                         long long* __restrict__ acc) {
    const TailStats ts = *tail;
    const int P = 2 * L.J + 4;
    long long r_mean = 0, l_mean = 0, r_tvar = 0, l_tvar = 0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const int64_t n = L.trial_count;
    // four trials per thread per round, their loads in flight together
    constexpr int kU = 4;
    for (int64_t k0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k0 < n; k0 += kU * stride) {
        double sv[kU], yv[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t k = k0 + u * stride;
            sv[u] = k < n ? S[k] : L.aggR;          // a trial past the end: ta = 0, no count
            yv[u] = k < n ? ylt[k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const double ta = sv[u] - L.aggR;
            const uint64_t key = __double_as_longlong(yv[u] + 0.0);
            const long long wt = key > ts.v_bits ? ts.c_eq : (key == ts.v_bits ? ts.m - ts.c_gt : 0);
            if ((ta > 0.0) && (ta < L.aggL)) {
                r_mean -= 1;
                r_tvar -= wt;
            }
            if (ta > L.aggL) {
                l_mean += 1;
                l_tvar += wt;
            }
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        r_mean += __shfl_xor(r_mean, off, kWave);
        l_mean += __shfl_xor(l_mean, off, kWave);
        r_tvar += __shfl_xor(r_tvar, off, kWave);
        l_tvar += __shfl_xor(l_tvar, off, kWave);
    }
    // one set of device atomics per workgroup: every workgroup adds to the
    // same four counters, so per-wave atomics would queue on them
    __shared__ long long red[4][4];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w][0] = r_mean;
        red[w][1] = l_mean;
        red[w][2] = r_tvar;
        red[w][3] = l_tvar;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long v[4] = {0, 0, 0, 0};
        for (int i = 0; i < static_cast<int>(blockDim.x >> 6); ++i)
            for (int q = 0; q < 4; ++q) v[q] += red[i][q];
        if (v[0]) add_i64(&acc[P - 2], v[0]);
        if (v[1]) add_i64(&acc[P - 1], v[1]);
        if (v[2]) add_i64(&acc[kMaxP + P - 2], v[2]);
        if (v[3]) add_i64(&acc[kMaxP + P - 1], v[3]);
    }
}

// g(E) W(E) over the catalogue; per-workgroup int64 accumulators in LDS
__global__ __launch_bounds__(256) void catalogue_kernel(const double* __restrict__ elts, int64_t C, LayerArgs L,
                                                        const uint64_t* __restrict__ w_mean,
                                                        const uint64_t* __restrict__ w_tvar,
                                                        long long* __restrict__ acc) {
    __shared__ long long lacc[2 * kMaxP];
    const int P = 2 * L.J + 4;
    for (int i = threadIdx.x; i < 2 * kMaxP; i += blockDim.x) lacc[i] = 0;
    __syncthreads();
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < C; e += stride) {
        const long long wm = static_cast<long long>(w_mean[e]);
        const long long wv = static_cast<long long>(w_tvar[e]);
        if (wm == 0 && wv == 0) continue;
        double y = 0.0;
        for (int j = 0; j < L.J; ++j)
            y = y + apply_terms(elts[static_cast<int64_t>(L.idx[j]) * C + e], L.R[j], L.Lim[j]);
        const double to = y - L.occR;
        const bool in_occ = (to > 0.0) && (to < L.occL);
        const bool above_occ = to > L.occL;
        if (above_occ) {
            add_i64(&lacc[2 * L.J + 1], wm);
            if (wv) add_i64(&lacc[kMaxP + 2 * L.J + 1], wv);
        }
        if (!in_occ) continue;
        add_i64(&lacc[2 * L.J], -wm);
        if (wv) add_i64(&lacc[kMaxP + 2 * L.J], -wv);
        for (int j = 0; j < L.J; ++j) {
            const double tj = elts[static_cast<int64_t>(L.idx[j]) * C + e] - L.R[j];
            if (tj > 0.0 && tj < L.Lim[j]) {
                add_i64(&lacc[j], -wm);
                if (wv) add_i64(&lacc[kMaxP + j], -wv);
            }
            if (tj > L.Lim[j]) {
                add_i64(&lacc[L.J + j], wm);
                if (wv) add_i64(&lacc[kMaxP + L.J + j], wv);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * kMaxP; i += blockDim.x) {
        const int q = i % kMaxP;
        if (q < P - 2 && lacc[i] != 0) add_i64(&acc[i], lacc[i]);
    }
}

__global__ void finalize_kernel(const long long* acc, const TailStats* tail, int P, int64_t n,
                                double* grad_mean, double* grad_tvar) {
    const int i = threadIdx.x;
    if (i >= P) return;
    const TailStats ts = *tail;
    if (grad_mean) grad_mean[i] = static_cast<double>(acc[i]) / static_cast<double>(n);
    if (grad_tvar) grad_tvar[i] = static_cast<double>(acc[kMaxP + i]) / static_cast<double>(ts.m * ts.c_eq);
}

AdjScratch carve(void* base, int64_t C, int64_t n) {
    char* p = static_cast<char*>(base);
    AdjScratch s;
    const int64_t Ca = (C + 255) & ~int64_t(255);
    s.w_mean = reinterpret_cast<uint64_t*>(p);
    p += Ca * sizeof(uint64_t);
    s.w_tvar = reinterpret_cast<uint64_t*>(p);
    p += Ca * sizeof(uint64_t);
    s.acc = reinterpret_cast<long long*>(p);
    p += 2 * kMaxP * sizeof(long long);
    s.tail = reinterpret_cast<TailStats*>(p);
    p += 256;
    s.mark = reinterpret_cast<uint8_t*>(p);
    p += Ca;
    s.cls = p;
    s.cls_bytes = (stream_adjoint_scratch_bytes(n) + 255) & ~int64_t(255);
    p += s.cls_bytes;
    s.tail_scratch = p;
    return s;
}

}  // namespace

int64_t adjoint_scratch_bytes(int64_t C, int J, int64_t n) {
    (void)J;
    const int64_t Ca = (C + 255) & ~int64_t(255);
    return Ca * (2 * sizeof(uint64_t) + 1) + 2 * kMaxP * sizeof(long long) + 256 +
           ((stream_adjoint_scratch_bytes(n) + 255) & ~int64_t(255)) + tail_stats_scratch_bytes(n);
}

hipError_t launch_adjoint(const int64_t* offsets, const uint32_t* ids, const double* elts, int64_t C,
                          const LayerArgs& L, const double* S, const double* ylt, int64_t m, void* scratch,
                          double* d_grad_mean, double* d_grad_tvar, int n_cu, hipStream_t s,
                          const PartLayout* parts, void* part_scratch, int64_t n_trials_total,
                          const SparsePool* sp, const StreamLayout* stream) {
    AdjScratch a = carve(scratch, C, L.trial_count);
    hipError_t err;
    const int64_t n = L.trial_count;
    if ((err = launch_tail_stats(ylt, n, m, a.tail_scratch, a.tail, n_cu, s)) != hipSuccess) return err;
    hipLaunchKernelGGL(clear_acc_kernel, dim3(1), dim3(256), 0, s, a.acc);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    const uint32_t cblocks = static_cast<uint32_t>((C + 255) / 256);
    const int with_mark = (parts && parts->P > 0 && part_scratch) ? 0 : 1;
    hipLaunchKernelGGL(mark_kernel, dim3(cblocks), dim3(256), 0, s, elts, C, L, a.mark, a.w_mean, a.w_tvar,
                       with_mark);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if (parts && parts->P > 0 && part_scratch) {
        int64_t ab = (n + 255) / 256;
        if (ab > int64_t(n_cu)) ab = int64_t(n_cu);
        if (ab < 1) ab = 1;
        hipLaunchKernelGGL(agg_counts_kernel, dim3(static_cast<uint32_t>(ab)), dim3(256), 0, s, L, S, ylt, a.tail,
                           a.acc);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        if (stream && stream->P > 0 && (stream->P - 1) / 4 < parts->P) {
            if ((err = launch_stream_adjoint(*stream, C, L, part_scratch, parts->P, S, ylt, a.tail, a.cls,
                                             a.cls_bytes, a.w_mean, a.w_tvar, n_cu, s)) != hipSuccess)
                return err;
        } else if ((err = launch_part_adjoint(*parts, n_trials_total, L, part_scratch, S, ylt, a.tail, a.w_mean,
                                              a.w_tvar, n_cu, s)) != hipSuccess) {
            return err;
        }
    } else {
        int64_t tblocks = (n + 3) / 4;
        if (tblocks > int64_t(n_cu) * 8) tblocks = int64_t(n_cu) * 8;
        if (tblocks < 1) tblocks = 1;
        hipLaunchKernelGGL(active_trials_kernel, dim3(static_cast<uint32_t>(tblocks)), dim3(256), 0, s, offsets,
                           ids, L, S, ylt, a.tail, a.mark, a.w_mean, a.w_tvar, a.acc);
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    if (sp && sp->chunk_off && sp->n_chunks == (C + kSparseChunk - 1) / kSparseChunk) {
        hipLaunchKernelGGL(catalogue_sparse_kernel, dim3(static_cast<uint32_t>(sp->n_chunks)), dim3(1024), 0, s, *sp,
                           C, L, a.w_mean, a.w_tvar, a.acc);
    } else {
        int64_t gblocks = (C + 255) / 256;
        if (gblocks > int64_t(n_cu) * 4) gblocks = int64_t(n_cu) * 4;
        hipLaunchKernelGGL(catalogue_kernel, dim3(static_cast<uint32_t>(gblocks)), dim3(256), 0, s, elts, C, L,
                           a.w_mean, a.w_tvar, a.acc);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, s, a.acc, a.tail, 2 * L.J + 4, n, d_grad_mean,
                       d_grad_tvar);
    return hipGetLastError();
}

}  // namespace ara
