// Program and portfolio year losses (Algorithm 1's outer loops, Section
// IV-A): per trial, the sum of the year losses of a program's layers, and
// of every layer of the portfolio.
//
// The layers' YLTs lie row by row ([layer][trial]), so a thread per trial
// reads one double per layer with consecutive threads on consecutive
// addresses: every read is a fully used 64-byte segment per quarter wave,
// and the pass moves (n_layers + n_programs + 1) x 8 bytes per trial, bound
// by HBM bandwidth.  Sums are double-double in layer order, rounded once.
#include "ara_internal.hpp"

namespace ara {

namespace {

constexpr int kSumThreads = 256;
constexpr int kLoadsInFlight = 4;   // layer reads issued before their sums

__global__ __launch_bounds__(kSumThreads) void portfolio_sum_kernel(PortfolioSumArgs a) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < a.count; k += stride) {
        double fh = 0.0, fl = 0.0;
        for (int p = 0; p < a.n_programs; ++p) {
            double ph = 0.0, pl = 0.0;
            const int l1 = a.first[p + 1];
            for (int l = a.first[p]; l < l1; l += kLoadsInFlight) {
                double v[kLoadsInFlight];
#pragma unroll
                for (int u = 0; u < kLoadsInFlight; ++u)
                    v[u] = l + u < l1 ? a.layer_ylt[static_cast<int64_t>(l + u) * a.count + k] : 0.0;
#pragma unroll
                for (int u = 0; u < kLoadsInFlight; ++u)
                    if (l + u < l1) dd_add(ph, pl, v[u]);
            }
            if (a.program_ylt) a.program_ylt[static_cast<int64_t>(p) * a.count + k] = ph + pl;
            dd_merge(fh, fl, ph, pl);
        }
        if (a.portfolio_ylt) a.portfolio_ylt[k] = fh + fl;
    }
}

}  // namespace

hipError_t launch_portfolio_sum(const PortfolioSumArgs& a, int n_cu, hipStream_t s) {
    if (a.count <= 0) return hipSuccess;
    int64_t blocks = (a.count + kSumThreads - 1) / kSumThreads;
    const int64_t cap = static_cast<int64_t>(n_cu) * 16;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(portfolio_sum_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(kSumThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace ara
