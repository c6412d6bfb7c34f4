// Trial-pass kernels: Algorithm 3 of the paper on gfx950.
//
// Two ways to evaluate one occurrence's loss o(E):
//  * literal  -- for every occurrence, look E up in each of the layer's ELTs,
//                apply the ELT terms, sum in layer order, apply the occurrence
//                terms (Algorithm 3 as written);
//  * folded   -- o depends on the event ID only (the occurrence terms apply to
//                each occurrence independently of the others), so a fold
//                kernel evaluates it once per catalogue event with the same
//                FP64 operations in the same order, and the trial pass does a
//                single gather o[E] per occurrence.  Bit-identical to literal.
//
// The trial pass streams the event IDs with non-temporal 16-byte loads (the
// YET is read once per run and must not evict the gather tables from L2),
// gathers o[E] (or the ELT losses), and accumulates the year's total in
// double-double so the rounded S is the correctly rounded sum of the
// occurrence losses (up to ties within ~K u^2 S).  A group of LPT lanes owns
// one trial; LPT = 64 is a whole wavefront.
#include "ara_internal.hpp"

namespace ara {

namespace {

__device__ __forceinline__ u32x4 load_ids_nt(const uint32_t* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
}

// ---------------------------------------------------------------------------
// fold: o(E) for every catalogue event E
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void fold_kernel(const double* __restrict__ elts, int64_t C,
                                                   LayerArgs L, double* __restrict__ o) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= C) return;
    double y = 0.0;
    for (int j = 0; j < L.J; ++j) {
        const double l = elts[static_cast<int64_t>(L.idx[j]) * C + e];
        y = y + apply_terms(l, L.R[j], L.Lim[j]);
    }
    o[e] = apply_terms(y, L.occR, L.occL);
}

// ---------------------------------------------------------------------------
// trial pass
// ---------------------------------------------------------------------------

template <bool LITERAL>
__device__ __forceinline__ void occurrence_losses(const TrialPassArgs& a, const LayerArgs& L,
                                                  const u32x4 v, const bool valid[4],
                                                  double oq[4]) {
    if constexpr (LITERAL) {
        double y[4] = {0.0, 0.0, 0.0, 0.0};
        // ELT-outer over the lane's events: every lane of the wave reads the
        // same ELT at the same time, as the paper's kernel has a whole thread
        // block work on one ELT at once (Section IV-B); each event still sums
        // its ELTs in layer order.
        for (int j = 0; j < L.J; ++j) {
            const double* row = a.elts + static_cast<int64_t>(L.idx[j]) * a.C;
            const double R = L.R[j];
            const double Lim = L.Lim[j];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (valid[q]) y[q] = y[q] + apply_terms(row[v[q]], R, Lim);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) oq[q] = valid[q] ? apply_terms(y[q], L.occR, L.occL) : 0.0;
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) oq[q] = valid[q] ? a.o[v[q]] : 0.0;
    }
}

template <int LPT, bool LITERAL, bool CKPT>
__global__ __launch_bounds__(256) void trial_pass_kernel(TrialPassArgs a, LayerArgs L) {
    static_assert(LPT == 64 || LPT == 32 || LPT == 16 || LPT == 8, "lanes per trial");
    static_assert(!CKPT || LPT == 64, "checkpoints need a whole wave per trial");
    constexpr int64_t kChunk = LPT * 4;
    const int lig = threadIdx.x & (LPT - 1);
    int64_t group = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / LPT;
    const int64_t n_groups = (static_cast<int64_t>(gridDim.x) * blockDim.x) / LPT;
    if constexpr (LPT == 64) group = uniform_i64(group);

    for (int64_t k = group; k < L.trial_count; k += n_groups) {
        const int64_t t = L.trial_begin + k;
        const int64_t b = a.offsets[t];
        const int64_t e = a.offsets[t + 1];
        double hi = 0.0, lo = 0.0;
        const int64_t start = CKPT ? (b & ~int64_t(255)) : (b & ~int64_t(3));
        if constexpr (!CKPT) {
            // kU chunks per lane in flight before any lookup
            constexpr int kU = 4;
            for (int64_t c = start; c < e; c += kChunk * kU) {
                u32x4 v[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int64_t base = c + u * kChunk + lig * 4;
                    v[u] = base < e ? load_ids_nt(a.ids + base) : u32x4{0u, 0u, 0u, 0u};
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int64_t base = c + u * kChunk + lig * 4;
                    bool valid[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) valid[q] = (base + q >= b) && (base + q < e);
                    double oq[4];
                    occurrence_losses<LITERAL>(a, L, v[u], valid, oq);
#pragma unroll
                    for (int q = 0; q < 4; ++q) dd_add(hi, lo, oq[q]);
                }
            }
        }
        for (int64_t c = start; CKPT && c < e; c += kChunk) {
            const int64_t base = c + lig * 4;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (base < e) v = load_ids_nt(a.ids + base);
            bool valid[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) valid[q] = (base + q >= b) && (base + q < e);
            double oq[4];
            occurrence_losses<LITERAL>(a, L, v, valid, oq);
            if constexpr (!CKPT) {
#pragma unroll
                for (int q = 0; q < 4; ++q) dd_add(hi, lo, oq[q]);
            } else {
                // lanes 16g..16g+15 hold global 64-event block c/64 + g
                double ph = 0.0, pl = 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q) dd_add(ph, pl, oq[q]);
                group_reduce_dd(ph, pl, 16);
                double th[4], tl[4];
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    th[g] = shfl_f64(ph, 16 * g);
                    tl[g] = shfl_f64(pl, 16 * g);
                }
                const int my = lig >> 4;
                double rh = hi, rl = lo;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    if (g <= my) dd_merge(rh, rl, th[g], tl[g]);
                }
                const int64_t blk = c / kStride + my;
                const int64_t last = blk * kStride + (kStride - 1);
                if ((lig & 15) == 0 && last >= b && last < e) a.stride[blk] = rh + rl;
#pragma unroll
                for (int g = 0; g < 4; ++g) dd_merge(hi, lo, th[g], tl[g]);
            }
        }
        if constexpr (!CKPT) group_reduce_dd(hi, lo, LPT);
        if (lig == 0) {
            const double S = hi + lo;
            a.ylt[k] = apply_terms(S, L.aggR, L.aggL);
            if (a.S) a.S[k] = S;
        }
    }
}

// ---------------------------------------------------------------------------
// debug lookups, validation, fill
// ---------------------------------------------------------------------------

__global__ void debug_lookups_kernel(const int64_t* offsets, const uint32_t* ids, const double* elts,
                                     int64_t C, LayerArgs L, int64_t trial, uint32_t* ids_out,
                                     double* losses_out) {
    const int64_t b = offsets[trial];
    const int64_t e = offsets[trial + 1];
    for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
        const uint32_t id = ids[i];
        ids_out[i - b] = id;
        for (int j = 0; j < L.J; ++j)
            losses_out[(i - b) * L.J + j] = elts[static_cast<int64_t>(L.idx[j]) * C + id];
    }
}

// flags: bit 0 = ID out of range, bit 1 = offsets decrease, bit 2 = bad loss
__global__ void validate_kernel(const int64_t* offsets, int64_t n_trials, const uint32_t* ids,
                                int64_t n_events, const double* elts, int64_t n_vals, int64_t C,
                                uint32_t* flags) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    uint32_t f = 0;
    // the IDs 16 bytes at a time (the allocation is 256-byte aligned), then the tail
    const int64_t n4 = n_events / 4;
    const u32x4* ids4 = reinterpret_cast<const u32x4*>(ids);
    const uint32_t c32 = C > 0xFFFFFFFFll ? 0xFFFFFFFFu : static_cast<uint32_t>(C);
    const bool wide = C > 0xFFFFFFFFll;              // every 32-bit ID is below C
    for (int64_t i = tid; i < n4; i += stride) {
        const u32x4 v = __builtin_nontemporal_load(ids4 + i);
        if (!wide && (v.x >= c32 || v.y >= c32 || v.z >= c32 || v.w >= c32)) f |= 1u;
    }
    for (int64_t i = 4 * n4 + tid; i < n_events; i += stride)
        if (static_cast<int64_t>(ids[i]) >= C) f |= 1u;
    for (int64_t i = tid; i < n_trials; i += stride)
        if (offsets[i + 1] < offsets[i]) f |= 2u;
    for (int64_t i = tid; i < n_vals; i += stride) {
        const double v = elts[i];
        if (!(v >= 0.0) || __builtin_isinf(v)) f |= 4u;
    }
    if (f) atomicOr(flags, f);
}

__global__ void fill_kernel(double* p, int64_t n, double v) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = v;
}

template <int LPT, bool LITERAL, bool CKPT>
hipError_t launch_tp(const TrialPassArgs& a, const LayerArgs& L, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((trial_pass_kernel<LPT, LITERAL, CKPT>), dim3(blocks), dim3(256), 0, s, a, L);
    return hipGetLastError();
}

template <bool LITERAL>
hipError_t launch_tp_lpt(const TrialPassArgs& a, const LayerArgs& L, int lpt, bool ckpt,
                         int blocks, hipStream_t s) {
    if (ckpt) return launch_tp<64, LITERAL, true>(a, L, blocks, s);
    switch (lpt) {
        case 8: return launch_tp<8, LITERAL, false>(a, L, blocks, s);
        case 16: return launch_tp<16, LITERAL, false>(a, L, blocks, s);
        case 32: return launch_tp<32, LITERAL, false>(a, L, blocks, s);
        default: return launch_tp<64, LITERAL, false>(a, L, blocks, s);
    }
}

}  // namespace

hipError_t launch_fold(const double* elts, int64_t C, const LayerArgs& L, double* o,
                       const ara_tuning& tu, hipStream_t s) {
    (void)tu;
    if (C <= 0) return hipSuccess;
    const int64_t blocks = (C + 255) / 256;
    hipLaunchKernelGGL(fold_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, elts, C, L, o);
    return hipGetLastError();
}

hipError_t launch_trial_pass(const TrialPassArgs& a, const LayerArgs& L, bool literal,
                             const ara_tuning& tu, int n_cu, hipStream_t s) {
    if (L.trial_count <= 0) return hipSuccess;
    int lpt = tu.lanes_per_trial > 0 ? tu.lanes_per_trial : 64;
    const bool ckpt = a.stride != nullptr;
    if (ckpt) lpt = 64;
    const int per_cu = tu.blocks_per_cu > 0 ? tu.blocks_per_cu : 8;
    const int64_t groups_per_block = 256 / lpt;
    int64_t blocks = (L.trial_count + groups_per_block - 1) / groups_per_block;
    const int64_t cap = static_cast<int64_t>(n_cu) * per_cu;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    return literal ? launch_tp_lpt<true>(a, L, lpt, ckpt, static_cast<int>(blocks), s)
                   : launch_tp_lpt<false>(a, L, lpt, ckpt, static_cast<int>(blocks), s);
}

hipError_t launch_debug_lookups(const int64_t* offsets, const uint32_t* ids, const double* elts,
                                int64_t C, const LayerArgs& L, int64_t trial, uint32_t* ids_out,
                                double* losses_out, hipStream_t s) {
    hipLaunchKernelGGL(debug_lookups_kernel, dim3(1), dim3(256), 0, s, offsets, ids, elts, C, L, trial,
                       ids_out, losses_out);
    return hipGetLastError();
}

hipError_t launch_validate(const int64_t* offsets, int64_t n_trials, const uint32_t* ids,
                           int64_t n_events, const double* elts, int64_t n_elt_values, int64_t C,
                           uint32_t* d_flags, int n_cu, hipStream_t s) {
    const int blocks = n_cu * 8;                 // 32 waves per CU
    hipLaunchKernelGGL(validate_kernel, dim3(blocks), dim3(256), 0, s, offsets, n_trials, ids, n_events,
                       elts, n_elt_values, C, d_flags);
    return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace ara
