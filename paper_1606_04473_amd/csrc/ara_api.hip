// C ABI of libara: argument checks, table residency, the library's device
// memory cache, kernel dispatch.  No exception crosses the ABI.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <charconv>
#include <cstdlib>
#include <list>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "ara_internal.hpp"

// ---------------------------------------------------------------------------
// Device memory of the library.  Blocks come from hipMalloc in size classes
// (four per octave, so a block exceeds its request by under 25%) and are kept
// when freed: a freed block is handed out again at once for work on the
// stream that freed it (stream order covers the earlier use), and for work on
// any other stream once an event recorded at the free has completed, which
// is checked without waiting.  In steady state no call allocates from or
// returns memory to the runtime, so independent streams never wait on each
// other inside an allocation.  Idle blocks are released (hipFree) only when
// hipMalloc runs out of memory.
namespace ara {
namespace {

struct CacheBlock {
    size_t size = 0;
    hipStream_t stream = nullptr;   // stream of the last free
    hipEvent_t ready = nullptr;     // recorded on it at that free
    bool in_use = true;
};

struct DeviceCache {
    std::mutex mu;
    std::unordered_map<void*, CacheBlock> blocks;
};

DeviceCache& device_cache(int device) {
    static std::mutex mu;
    static std::vector<std::pair<int, DeviceCache*>> caches;     // kept until the process ends
    std::lock_guard<std::mutex> g(mu);
    for (auto& c : caches)
        if (c.first == device) return *c.second;
    caches.emplace_back(device, new DeviceCache());
    return *caches.back().second;
}

size_t size_class(size_t bytes) {
    if (bytes <= 512) return 512;
    const int k = 63 - __builtin_clzll(static_cast<unsigned long long>(bytes));
    const size_t base = size_t(1) << k;             // base <= bytes < 2 base
    const size_t step = base >> 2;
    return base + (bytes - base + step - 1) / step * step;
}

// hipFree of the idle blocks whose last free has completed, or that have no
// event (hipFree waits for the device); returns the bytes released
int64_t release_idle(DeviceCache& c) {
    std::lock_guard<std::mutex> g(c.mu);
    int64_t freed = 0;
    for (auto it = c.blocks.begin(); it != c.blocks.end();) {
        CacheBlock& b = it->second;
        if (!b.in_use && (!b.ready || hipEventQuery(b.ready) == hipSuccess)) {
            if (b.ready) (void)hipEventDestroy(b.ready);
            (void)hipFree(it->first);
            freed += static_cast<int64_t>(b.size);
            it = c.blocks.erase(it);
        } else {
            ++it;
        }
    }
    return freed;
}

}  // namespace

void cache_stats(int device, int64_t* held, int64_t* idle) {
    DeviceCache& c = device_cache(device);
    std::lock_guard<std::mutex> g(c.mu);
    int64_t h = 0, i = 0;
    for (auto& kv : c.blocks) {
        h += static_cast<int64_t>(kv.second.size);
        if (!kv.second.in_use) i += static_cast<int64_t>(kv.second.size);
    }
    *held = h;
    *idle = i;
}

int64_t cache_release(int device) { return release_idle(device_cache(device)); }

hipError_t dev_alloc(void** p, size_t bytes, hipStream_t s) {
    *p = nullptr;
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return e;
    DeviceCache& c = device_cache(device);
    const size_t cls = size_class(bytes);
    {
        std::lock_guard<std::mutex> g(c.mu);
        for (auto& kv : c.blocks) {
            CacheBlock& b = kv.second;
            if (b.in_use || b.size != cls) continue;
            // another stream only once the free is known to be complete (a
            // block without an event serves its own stream only)
            if (b.stream != s && (!b.ready || hipEventQuery(b.ready) != hipSuccess)) continue;
            b.in_use = true;
            *p = kv.first;
            return hipSuccess;
        }
    }
    void* q = nullptr;
    e = hipMalloc(&q, cls);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        release_idle(c);
        e = hipMalloc(&q, cls);
    }
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> g(c.mu);
    CacheBlock b;
    b.size = cls;
    b.stream = s;
    c.blocks.emplace(q, b);
    *p = q;
    return hipSuccess;
}

void dev_free(void* p, hipStream_t s) {
    if (!p) return;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return;
    DeviceCache& c = device_cache(device);
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.blocks.find(p);
    if (it == c.blocks.end()) return;
    CacheBlock& b = it->second;
    if (!b.ready && hipEventCreateWithFlags(&b.ready, hipEventDisableTiming) != hipSuccess) b.ready = nullptr;
    if (b.ready && hipEventRecord(b.ready, s) != hipSuccess) {
        // without an event the block can only go back to work on s
        (void)hipEventDestroy(b.ready);
        b.ready = nullptr;
    }
    b.stream = s;
    b.in_use = false;
}

}  // namespace ara

namespace {

thread_local std::string g_error;

ara_status fail(ara_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return st;
}

ara_status hip_fail(hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(ARA_ERR_NO_MEMORY, "%s: %s", what, hipGetErrorString(e));
    return fail(ARA_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                       \
    do {                                          \
        hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// Make the tables' device current for the scope of a call.
struct DeviceScope {
    int prev = -1;
    bool ok = true;
    explicit DeviceScope(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceScope() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Stream-ordered scratch that is returned to the pool when the scope ends.
struct PoolBuffer {
    void* p = nullptr;
    hipStream_t s = nullptr;
    ~PoolBuffer() {
        if (p) ara::dev_free(p, s);
    }
    hipError_t alloc(size_t bytes, hipStream_t stream) {
        s = stream;
        if (bytes == 0) bytes = 256;
        return ara::dev_alloc(&p, bytes, stream);
    }
};

// Take a kept scratch buffer of at least `bytes` for work on stream s (see
// ScratchBuffer); give it back with scratch_release after enqueueing.
hipError_t scratch_acquire(std::mutex& mu, std::vector<ara::ScratchBuffer*>& sets, size_t bytes, hipStream_t s,
                           ara::ScratchBuffer** out) {
    *out = nullptr;
    ara::ScratchBuffer* pick = nullptr;
    {
        std::lock_guard<std::mutex> g(mu);
        for (auto* b : sets) {
            if (b->busy) continue;
            if (b->stream != s && b->done && hipEventQuery(b->done) != hipSuccess) continue;
            if (!pick || (b->cap >= bytes && (pick->cap < bytes || b->stream == s))) pick = b;
        }
        if (!pick) {
            pick = new (std::nothrow) ara::ScratchBuffer();
            if (!pick) return hipErrorOutOfMemory;
            sets.push_back(pick);
        }
        pick->busy = true;
    }
    hipError_t e = hipSuccess;
    if (!pick->done) e = hipEventCreateWithFlags(&pick->done, hipEventDisableTiming);
    if (e == hipSuccess && pick->cap < bytes) {
        // growing: the old memory may still be read by work on its last
        // stream, so it goes back to the cache in that stream's order; the new
        // memory is taken in this call's stream order
        if (pick->p) ara::dev_free(pick->p, pick->stream);
        pick->p = nullptr;
        pick->cap = 0;
        pick->primed = false;
        if (e == hipSuccess) e = ara::dev_alloc(&pick->p, bytes, s);
        if (e == hipSuccess) pick->cap = bytes;
    }
    if (e != hipSuccess) {
        std::lock_guard<std::mutex> g(mu);
        pick->busy = false;
        return e;
    }
    *out = pick;
    return hipSuccess;
}

void scratch_release(std::mutex& mu, ara::ScratchBuffer* b, hipStream_t s) {
    if (!b) return;
    (void)hipEventRecord(b->done, s);
    std::lock_guard<std::mutex> g(mu);
    b->stream = s;
    b->busy = false;
}

// frees on stream fs after each buffer's last use (its event)
void scratch_free_all(std::vector<ara::ScratchBuffer*>& sets, hipStream_t fs) {
    for (auto* b : sets) {
        if (b->done) (void)hipStreamWaitEvent(fs, b->done, 0);
        if (b->p) ara::dev_free(b->p, fs);
        if (b->done) (void)hipEventDestroy(b->done);
        delete b;
    }
    sets.clear();
}

// the stream on which destroyed tables return their memory to the pool (one
// per device, default priority, never destroyed)
hipStream_t free_stream(int device) {
    static std::mutex mu;
    static std::vector<std::pair<int, hipStream_t>> streams;
    std::lock_guard<std::mutex> g(mu);
    for (auto& d : streams)
        if (d.first == device) return d.second;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
    streams.emplace_back(device, st);
    return st;
}

// Records, on stream s, an event after the work enqueued there so far on t's
// behalf (one event per stream, re-recorded by later calls).
void note_use(ara_tables* t, hipStream_t s) {
    std::lock_guard<std::mutex> g(t->fence_mu);
    for (auto& f : t->fences)
        if (f.first == s) {
            (void)hipEventRecord(f.second, s);
            return;
        }
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return;
    if (hipEventRecord(ev, s) != hipSuccess) {
        (void)hipEventDestroy(ev);
        return;
    }
    t->fences.emplace_back(s, ev);
}

// note_use on scope exit, so a call's error returns are covered too
struct UseFence {
    ara_tables* t;
    hipStream_t s;
    UseFence(ara_tables* tt, hipStream_t ss) : t(tt), s(ss) {}
    ~UseFence() {
        if (t) note_use(t, s);
    }
};

// releases on scope exit, so early error returns give the buffer back
struct ScratchLease {
    std::mutex& mu;
    ara::ScratchBuffer* b = nullptr;
    hipStream_t s = nullptr;
    ScratchLease(std::mutex& m) : mu(m) {}
    ~ScratchLease() { scratch_release(mu, b, s); }
};

bool bad_term(double v) { return std::isnan(v) || v < 0.0; }

ara_status build_layer_args(const ara_tables* t, const ara_layer& in, ara::LayerArgs& L) {
    std::memset(&L, 0, sizeof(L));
    if (in.n_elts < 0) return fail(ARA_ERR_INVALID_ARG, "layer n_elts < 0");
    if (in.n_elts > ara::kMaxJ)
        return fail(ARA_ERR_UNSUPPORTED, "layer covers %d ELTs; at most %d supported", in.n_elts, ara::kMaxJ);
    if (in.n_elts > 0 && (!in.elt_index || !in.elt_retention || !in.elt_limit))
        return fail(ARA_ERR_INVALID_ARG, "layer ELT arrays are NULL");
    L.J = in.n_elts;
    for (int j = 0; j < in.n_elts; ++j) {
        if (in.elt_index[j] < 0 || in.elt_index[j] >= t->n_pool)
            return fail(ARA_ERR_OUT_OF_RANGE, "ELT index %d outside the pool of %d", in.elt_index[j], t->n_pool);
        if (bad_term(in.elt_retention[j]) || bad_term(in.elt_limit[j]) || std::isinf(in.elt_retention[j]))
            return fail(ARA_ERR_INVALID_ARG, "ELT %d terms must be >= 0, finite retention, not NaN", j);
        L.idx[j] = in.elt_index[j];
        L.R[j] = in.elt_retention[j];
        L.Lim[j] = in.elt_limit[j];
    }
    if (bad_term(in.occ_retention) || bad_term(in.occ_limit) || bad_term(in.agg_retention) ||
        bad_term(in.agg_limit) || std::isinf(in.occ_retention) || std::isinf(in.agg_retention))
        return fail(ARA_ERR_INVALID_ARG, "layer terms must be >= 0, finite retentions, not NaN");
    L.occR = in.occ_retention;
    L.occL = in.occ_limit;
    L.aggR = in.agg_retention;
    L.aggL = in.agg_limit;
    if (in.trial_begin < 0 || in.trial_count < 0 || in.trial_begin > t->n_trials ||
        in.trial_count > t->n_trials - in.trial_begin)
        return fail(ARA_ERR_INVALID_ARG, "trial range [%lld, +%lld) outside [0, %lld)",
                    (long long)in.trial_begin, (long long)in.trial_count, (long long)t->n_trials);
    L.trial_begin = in.trial_begin;
    L.trial_count = in.trial_count;
    return ARA_OK;
}

bool same_layer(const ara::LayerArgs& a, const ara::LayerArgs& b) {
    if (a.J != b.J || a.trial_begin != b.trial_begin || a.trial_count != b.trial_count) return false;
    if (a.occR != b.occR || a.occL != b.occL || a.aggR != b.aggR || a.aggL != b.aggL) return false;
    for (int j = 0; j < a.J; ++j)
        if (a.idx[j] != b.idx[j] || a.R[j] != b.R[j] || a.Lim[j] != b.Lim[j]) return false;
    return true;
}

// m = ceil(n (1 - p)) with p read as the decimal it was written as: the
// shortest decimal string that converts back to the same double (what
// std::to_chars produces), taken exactly.  With that string's digits D and
// k decimal places, p = D / 10^k and m = n - floor(n D / 10^k), clamped to
// [1, n].  n D < 2^63 * 10^17 < 2^120 fits in 128 bits; for k > 38 the
// quotient is 0.  Requires 1 <= n and 0 < p < 1.
int64_t tail_count(int64_t n, double p) {
    char buf[64];
    const auto r = std::to_chars(buf, buf + sizeof(buf), p, std::chars_format::scientific);
    *r.ptr = '\0';
    // "d.ddde-XX" or "de-XX": mantissa digits, then the exponent
    unsigned __int128 D = 0;
    int nd = 0;
    const char* c = buf;
    for (; *c && *c != 'e'; ++c) {
        if (*c == '.') continue;
        D = D * 10u + static_cast<unsigned>(*c - '0');
        ++nd;
    }
    const int e10 = (*c == 'e') ? std::atoi(c + 1) : 0;
    const int k = (nd - 1) - e10;                   // p = D * 10^-k, k >= 1 since p < 1
    unsigned __int128 q = 0;
    if (k <= 38) {
        unsigned __int128 pow10 = 1;
        for (int i = 0; i < k; ++i) pow10 *= 10u;
        q = (static_cast<unsigned __int128>(static_cast<uint64_t>(n)) * D) / pow10;
    }
    int64_t m = n - static_cast<int64_t>(q);
    if (m < 1) m = 1;
    if (m > n) m = n;
    return m;
}

void free_checkpoints(ara::CheckpointState& ck) {
    if (ck.S) (void)hipFree(ck.S);
    if (ck.ylt) (void)hipFree(ck.ylt);
    if (ck.stride) (void)hipFree(ck.stride);
    ck = ara::CheckpointState{};
}

hipError_t take_event(ara::ProfileState& ps, hipEvent_t* ev) {
    if (!ps.free_events.empty()) {
        *ev = ps.free_events.back();
        ps.free_events.pop_back();
        return hipSuccess;
    }
    // timing only: no system-scope fence on record, which would write back and
    // invalidate the caches between the kernels being timed
    return hipEventCreateWithFlags(ev, hipEventDisableSystemFence);
}

// Records an event pair around a launch when profiling is on.
struct KernelTimer {
    ara_tables* t;
    hipStream_t s;
    bool on;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    KernelTimer(ara_tables* t_, hipStream_t s_, bool on_, int kind_) : t(t_), s(s_), on(on_), kind(kind_) {
        if (!on) return;
        std::lock_guard<std::mutex> g(t->prof_mu);
        if (take_event(t->prof, &a) != hipSuccess || take_event(t->prof, &b) != hipSuccess) {
            on = false;
            return;
        }
        if (hipEventRecord(a, s) != hipSuccess) on = false;
    }
    void done() {
        if (!on) return;
        if (hipEventRecord(b, s) != hipSuccess) return;
        std::lock_guard<std::mutex> g(t->prof_mu);
        t->prof.pending.push_back({a, b, kind});
        on = false;
    }
};

// Make the staging buffer at least `bytes` and wait for earlier copies out of it.
hipError_t stage_acquire(ara::HostStage& st, size_t bytes) {
    hipError_t e;
    if (!st.done && (e = hipEventCreateWithFlags(&st.done, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventSynchronize(st.done)) != hipSuccess) return e;
    if (st.cap < bytes) {
        if (st.p) (void)hipHostFree(st.p);
        st.p = nullptr;
        st.cap = 0;
        size_t want = bytes < (1u << 20) ? (1u << 20) : bytes;
        if ((e = hipHostMalloc(&st.p, want, hipHostMallocDefault)) != hipSuccess) return e;
        st.cap = want;
    }
    return hipSuccess;
}

// Copy a graph's layer arguments to the head of its scratch through its pinned
// stage.  Arguments equal to the last ones copied are already there -- in
// stream order on the stream that copied them, on any stream once that copy
// has completed -- so nothing is copied and the host does not wait for the
// stage: a caller that replays a graph with the same terms can queue many
// replays ahead of the device.
hipError_t upload_layer_args(ara::GraphEntry* e, const void* args, size_t bytes, hipStream_t s) {
    if (e->last.size() == bytes && std::memcmp(e->last.data(), args, bytes) == 0 &&
        (e->last_stream == s || hipEventQuery(e->stage.done) == hipSuccess))
        return hipSuccess;
    e->last.clear();
    hipError_t r = stage_acquire(e->stage, bytes);
    if (r != hipSuccess) return r;
    std::memcpy(e->stage.p, args, bytes);
    if ((r = hipMemcpyAsync(e->scratch, e->stage.p, bytes, hipMemcpyHostToDevice, s)) != hipSuccess) return r;
    if ((r = hipEventRecord(e->stage.done, s)) != hipSuccess) return r;
    const uint8_t* a = static_cast<const uint8_t*>(args);
    e->last.assign(a, a + bytes);
    e->last_stream = s;
    return hipSuccess;
}

void stage_free(ara::HostStage& st) {
    if (st.done) {
        (void)hipEventSynchronize(st.done);
        (void)hipEventDestroy(st.done);
    }
    if (st.p) (void)hipHostFree(st.p);
    st = ara::HostStage{};
}

void free_graph(ara::GraphEntry* g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    stage_free(g->stage);
    if (g->scratch) (void)hipFree(g->scratch);
    delete g;
}

// Host-side description of a batched run.
struct BatchPlan {
    std::vector<ara::BatchLayerDesc> layers;
    std::vector<ara::BatchFoldDesc> fold;
    std::vector<int32_t> idx;
    std::vector<double> R, Lim;
    std::vector<int2> items;
    std::vector<int64_t> key;
};

BatchPlan make_plan(const ara_tables* t, const std::vector<ara::LayerArgs>& L, const double* ylt_ptr,
                    int schedule) {
    BatchPlan b;
    const int T = t->parts.T;
    struct Cost {
        int64_t c;
        int l;
        int64_t tile;
    };
    std::vector<Cost> costs;
    b.key.push_back(static_cast<int64_t>(L.size()));
    b.key.push_back(reinterpret_cast<int64_t>(ylt_ptr));
    for (size_t l = 0; l < L.size(); ++l) {
        const auto& a = L[l];
        b.layers.push_back({a.trial_begin, a.trial_begin + a.trial_count, a.aggR, a.aggL, a.out_offset});
        b.fold.push_back({a.J, static_cast<int32_t>(b.idx.size()), a.occR, a.occL});
        for (int j = 0; j < a.J; ++j) {
            b.idx.push_back(a.idx[j]);
            b.R.push_back(a.R[j]);
            b.Lim.push_back(a.Lim[j]);
        }
        b.key.push_back(a.J);
        b.key.push_back(a.trial_begin);
        b.key.push_back(a.trial_count);
        if (a.trial_count <= 0) continue;
        const int64_t lo = a.trial_begin, hi = a.trial_begin + a.trial_count;
        for (int64_t tile = lo / T; tile * T < hi; ++tile) {
            const int64_t a0 = std::max(lo, tile * T), a1 = std::min(hi, (tile + 1) * T);
            costs.push_back({a1 - a0, static_cast<int>(l), tile});
        }
    }
    // schedule 0: decreasing cost (longest items first); 1: layer-major order
    if (schedule == 0)
        std::stable_sort(costs.begin(), costs.end(), [](const Cost& x, const Cost& y) { return x.c > y.c; });
    b.key.push_back(schedule);
    b.items.reserve(costs.size());
    for (const auto& c : costs) b.items.push_back(make_int2(c.l, static_cast<int>(c.tile)));
    return b;
}

// Copy the plan's descriptors (and, with_items, the work list) into the
// device scratch through pinned staging, on stream s.
hipError_t upload_plan(ara::HostStage& st, const BatchPlan& b, const ara::BatchedScratch& bs, bool with_items,
                       hipStream_t s) {
    const size_t n1 = sizeof(ara::BatchLayerDesc) * b.layers.size();
    const size_t n2 = sizeof(ara::BatchFoldDesc) * b.fold.size();
    const size_t n3 = sizeof(double) * b.R.size();
    const size_t n4 = sizeof(int32_t) * b.idx.size();
    const size_t n5 = with_items ? sizeof(int2) * b.items.size() : 0;
    hipError_t e;
    if ((e = stage_acquire(st, n1 + n2 + 2 * n3 + n4 + n5 + 64)) != hipSuccess) return e;
    char* h = static_cast<char*>(st.p);
    size_t off = 0;
    auto put = [&](void* dst, const void* src, size_t n) -> hipError_t {
        if (n == 0) return hipSuccess;
        std::memcpy(h + off, src, n);
        hipError_t r = hipMemcpyAsync(dst, h + off, n, hipMemcpyHostToDevice, s);
        off += (n + 15) & ~size_t(15);
        return r;
    };
    if ((e = put(bs.layers, b.layers.data(), n1)) != hipSuccess) return e;
    if ((e = put(bs.fold, b.fold.data(), n2)) != hipSuccess) return e;
    if ((e = put(bs.R, b.R.data(), n3)) != hipSuccess) return e;
    if ((e = put(bs.Lim, b.Lim.data(), n3)) != hipSuccess) return e;
    if ((e = put(bs.idx, b.idx.data(), n4)) != hipSuccess) return e;
    if ((e = put(bs.items, b.items.data(), n5)) != hipSuccess) return e;
    return hipEventRecord(st.done, s);
}

// The passes that write per-(part, trial) partial sums for a merge: the
// streaming pass over the 16-bit part-major copy (default), or the XCD-affine
// pass over the 32-bit partitioned copy (pass_variant 2, or tables without
// the 16-bit copy).
struct SplitPass {
    const ara_tables* t;
    bool stream;
    SplitPass(const ara_tables* tt, const ara_tuning& tu) : t(tt), stream(tu.pass_variant == 0 && tt->stream.P > 0) {}
    size_t partial_bytes(int64_t trials) const {
        const int64_t n = trials > 0 ? trials : 1;
        return stream ? static_cast<size_t>(ara::stream_partials_bytes(t->stream, n))
                      : sizeof(double) * 2 * static_cast<size_t>(t->parts.P) * n;
    }
    hipError_t pass(const ara::LayerArgs& L, void* part_scratch, void* partials, hipStream_t s) const {
        if (stream) return ara::launch_stream_pass(t->stream, t->C, L, part_scratch, t->parts.P, partials, t->n_cu, s);
        return ara::launch_xcd_pass(t->parts, t->n_trials, t->C, L, part_scratch, static_cast<double*>(partials),
                                    t->n_cu, s);
    }
    hipError_t combine(const ara::LayerArgs& L, const ara::LayerArgs* L_dev, const void* partials, double* ylt,
                       double* S, hipStream_t s) const {
        if (stream) return ara::launch_stream_combine(t->stream, L, L_dev, partials, ylt, S, s);
        return ara::launch_xcd_combine(t->parts, L, L_dev, static_cast<const double*>(partials), ylt, S, s);
    }
};

int query_cu_count(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess || prop.multiProcessorCount <= 0) return 256;
    return prop.multiProcessorCount;
}

}  // namespace

extern "C" {

const char* ara_last_error(void) { return g_error.c_str(); }

const char* ara_status_string(ara_status s) {
    switch (s) {
        case ARA_OK: return "ARA_OK";
        case ARA_ERR_INVALID_ARG: return "ARA_ERR_INVALID_ARG";
        case ARA_ERR_OUT_OF_RANGE: return "ARA_ERR_OUT_OF_RANGE";
        case ARA_ERR_BUFFER_TOO_SMALL: return "ARA_ERR_BUFFER_TOO_SMALL";
        case ARA_ERR_NO_MEMORY: return "ARA_ERR_NO_MEMORY";
        case ARA_ERR_DEVICE: return "ARA_ERR_DEVICE";
        case ARA_ERR_NOT_READY: return "ARA_ERR_NOT_READY";
        case ARA_ERR_UNSUPPORTED: return "ARA_ERR_UNSUPPORTED";
        default: return "ARA_ERR_UNKNOWN";
    }
}

ara_status ara_tail_count(int64_t n_trials, double p, int64_t* m) {
    if (!m) return fail(ARA_ERR_INVALID_ARG, "m is NULL");
    if (n_trials < 1) return fail(ARA_ERR_INVALID_ARG, "n_trials < 1");
    if (!(p > 0.0 && p < 1.0)) return fail(ARA_ERR_INVALID_ARG, "p must lie in (0, 1)");
    *m = tail_count(n_trials, p);
    return ARA_OK;
}

ara_status ara_device_info(int32_t* n_cu, int32_t* device) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (n_cu) *n_cu = query_cu_count(dev);
    if (device) *device = dev;
    return ARA_OK;
}

static ara_status create_impl(const int64_t* trial_offsets, int64_t n_trials, const uint32_t* event_ids,
                              int64_t n_events, const double* elt_losses, int32_t n_elts, int64_t catalogue_size,
                              uint32_t flags, void* stream, const ara_tables* base, ara_tables** out);

ara_status ara_create_tables(const int64_t* trial_offsets, int64_t n_trials, const uint32_t* event_ids,
                             int64_t n_events, const double* elt_losses, int32_t n_elts,
                             int64_t catalogue_size, uint32_t flags, void* stream, ara_tables** out) {
    return create_impl(trial_offsets, n_trials, event_ids, n_events, elt_losses, n_elts, catalogue_size, flags,
                       stream, nullptr, out);
}

ara_status ara_create_yet(const ara_tables* base, const int64_t* trial_offsets, int64_t n_trials,
                          const uint32_t* event_ids, int64_t n_events, uint32_t flags, void* stream,
                          ara_tables** out) {
    if (!base) return fail(ARA_ERR_INVALID_ARG, "base tables are NULL");
    return create_impl(trial_offsets, n_trials, event_ids, n_events, base->elts, base->n_pool, base->C, flags,
                       stream, base, out);
}

static ara_status create_impl(const int64_t* trial_offsets, int64_t n_trials, const uint32_t* event_ids,
                              int64_t n_events, const double* elt_losses, int32_t n_elts, int64_t catalogue_size,
                              uint32_t flags, void* stream, const ara_tables* base, ara_tables** out) {
    if (!out) return fail(ARA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n_trials < 0 || n_events < 0 || n_elts < 0 || catalogue_size < 1)
        return fail(ARA_ERR_INVALID_ARG, "negative size or empty catalogue");
    if (catalogue_size >= (int64_t(1) << 32))
        return fail(ARA_ERR_INVALID_ARG, "catalogue of 2^32 events or more (IDs are uint32, 0xFFFFFFFF is reserved)");
    if (!trial_offsets || (n_events > 0 && !event_ids) || (n_elts > 0 && !elt_losses))
        return fail(ARA_ERR_INVALID_ARG, "NULL input array");
    const bool dev_in = (flags & ARA_DEVICE_PTR) != 0;
    if (!dev_in) {
        if (trial_offsets[0] != 0 || trial_offsets[n_trials] != n_events)
            return fail(ARA_ERR_INVALID_ARG, "offsets must start at 0 and end at n_events");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    int device = 0;
    if (base) {
        device = base->device;
        if (hipSetDevice(device) != hipSuccess) return fail(ARA_ERR_DEVICE, "cannot select the base tables' device");
    } else {
        HIP_TRY(hipGetDevice(&device), "hipGetDevice");
    }
    ara_tables* t = new (std::nothrow) ara_tables();
    if (!t) return fail(ARA_ERR_NO_MEMORY, "host allocation failed");
    t->device = device;
    t->n_cu = query_cu_count(device);
    t->n_trials = n_trials;
    t->n_events = n_events;
    t->C = catalogue_size;
    t->n_pool = n_elts;
    auto cleanup = [&](ara_status st) {
        note_use(t, s);                 // the memory goes back after the create's own work
        ara_destroy_tables(t);
        return st;
    };
    const size_t off_bytes = sizeof(int64_t) * (n_trials + 1);
    const size_t id_bytes = sizeof(uint32_t) * (n_events + ara::kIdPad);
    const size_t elt_bytes = base ? 0 : sizeof(double) * static_cast<size_t>(n_elts) * catalogue_size;
    if (base) {
        t->elts = const_cast<double*>(elt_losses);
        t->owns_elts = false;
        t->sparse = base->sparse;
        std::lock_guard<std::mutex> g(const_cast<ara_tables*>(base)->mu);
        t->tuning = base->tuning;
    }
    hipError_t e;
    if ((e = ara::dev_alloc(reinterpret_cast<void**>(&t->offsets), off_bytes, s)) != hipSuccess)
        return cleanup(hip_fail(e, "allocate offsets"));
    if ((e = ara::dev_alloc(reinterpret_cast<void**>(&t->ids), id_bytes, s)) != hipSuccess)
        return cleanup(hip_fail(e, "allocate event ids"));
    if (elt_bytes && (e = hipMalloc(&t->elts, elt_bytes)) != hipSuccess)
        return cleanup(hip_fail(e, "hipMalloc ELT pool"));
    t->bytes = static_cast<int64_t>(off_bytes + id_bytes + elt_bytes);
    const hipMemcpyKind kind = dev_in ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if ((e = hipMemcpyAsync(t->offsets, trial_offsets, off_bytes, kind, s)) != hipSuccess)
        return cleanup(hip_fail(e, "copy offsets"));
    if (n_events && (e = hipMemcpyAsync(t->ids, event_ids, sizeof(uint32_t) * n_events, kind, s)) != hipSuccess)
        return cleanup(hip_fail(e, "copy event ids"));
    if ((e = hipMemsetAsync(t->ids + n_events, 0, sizeof(uint32_t) * ara::kIdPad, s)) != hipSuccess)
        return cleanup(hip_fail(e, "clear id padding"));
    if (elt_bytes && (e = hipMemcpyAsync(t->elts, elt_losses, elt_bytes, kind, s)) != hipSuccess)
        return cleanup(hip_fail(e, "copy ELT pool"));
    // validation on the device, one flag word read back
    PoolBuffer flag;
    if ((e = flag.alloc(sizeof(uint32_t), s)) != hipSuccess) return cleanup(hip_fail(e, "scratch"));
    if ((e = hipMemsetAsync(flag.p, 0, sizeof(uint32_t), s)) != hipSuccess) return cleanup(hip_fail(e, "memset"));
    if ((e = ara::launch_validate(t->offsets, n_trials, t->ids, n_events, t->elts,
                                  base ? 0 : static_cast<int64_t>(n_elts) * catalogue_size, catalogue_size,
                                  static_cast<uint32_t*>(flag.p), t->n_cu, s)) != hipSuccess)
        return cleanup(hip_fail(e, "validate kernel"));
    uint32_t host_flag = 0;
    int64_t ends[2] = {0, 0};
    if ((e = hipMemcpyAsync(&host_flag, flag.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return cleanup(hip_fail(e, "read validation flag"));
    if ((e = hipMemcpyAsync(&ends[0], t->offsets, sizeof(int64_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(&ends[1], t->offsets + n_trials, sizeof(int64_t), hipMemcpyDeviceToHost, s)) !=
            hipSuccess)
        return cleanup(hip_fail(e, "read offsets"));
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return cleanup(hip_fail(e, "synchronize"));
    if (host_flag & 1u) return cleanup(fail(ARA_ERR_OUT_OF_RANGE, "an event ID is >= catalogue size %lld",
                                            (long long)catalogue_size));
    if ((host_flag & 2u) || ends[0] != 0 || ends[1] != n_events)
        return cleanup(fail(ARA_ERR_INVALID_ARG, "trial offsets must start at 0, not decrease, end at n_events"));
    if (host_flag & 4u) return cleanup(fail(ARA_ERR_INVALID_ARG, "ELT losses must be finite and >= 0"));
    if (!base) {
        // the pool's nonzero entries, which the per-request fold reads
        if ((e = ara::build_sparse_pool(t->elts, n_elts, catalogue_size, s, &t->sparse)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return cleanup(hip_fail(e, "sparse ELT pool"));
        t->bytes += t->sparse.bytes;
    }
    if (!(flags & ARA_PLAIN_LAYOUT) && n_trials > 0) {
        e = ara::build_part_layout(t->offsets, t->ids, n_trials, n_events, catalogue_size, t->n_cu, s, &t->parts);
        if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
            (void)hipGetLastError();
            t->parts = ara::PartLayout{};      // not enough memory for the copy: plain layout only
        } else if (e != hipSuccess) {
            return cleanup(hip_fail(e, "partitioned layout"));
        }
        t->bytes += t->parts.bytes;
        e = ara::build_stream_layout(t->offsets, t->ids, n_trials, n_events, catalogue_size, t->n_cu, s, &t->stream);
        if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
            (void)hipGetLastError();
            t->stream = ara::StreamLayout{};   // not enough memory for the 16-bit copy: 32-bit passes only
        } else if (e != hipSuccess) {
            return cleanup(hip_fail(e, "16-bit stream layout"));
        }
        t->bytes += t->stream.bytes;
    }
    note_use(t, s);
    *out = t;
    return ARA_OK;
}

void ara_destroy_tables(ara_tables* t) {
    if (!t) return;
    DeviceScope ds(t->device);
    // The YET, its layouts and the kept scratch come from the library's
    // device memory cache: they go back to it on an internal stream once every
    // stream the tables were used on has reached the end of its last call's
    // work, and the host does not wait (a hipFree would wait for the whole
    // device)
    hipStream_t fs = free_stream(t->device);
    {
        std::lock_guard<std::mutex> g(t->fence_mu);
        for (auto& f : t->fences) {
            (void)hipStreamWaitEvent(fs, f.second, 0);
            (void)hipEventDestroy(f.second);
        }
        t->fences.clear();
    }
    if (t->offsets) ara::dev_free(t->offsets, fs);
    if (t->ids) ara::dev_free(t->ids, fs);
    scratch_free_all(t->scratch, fs);
    ara::free_part_layout(&t->parts, fs);
    ara::free_stream_layout(&t->stream, fs);
    if (t->elts && t->owns_elts) (void)hipFree(t->elts);
    if (t->owns_elts) ara::free_sparse_pool(&t->sparse);
    free_checkpoints(t->ck);
    for (auto* g : t->graphs) free_graph(g);
    t->graphs.clear();
    stage_free(t->stage);
    for (auto& p : t->prof.pending) {
        (void)hipEventDestroy(p.start);
        (void)hipEventDestroy(p.stop);
    }
    for (auto e : t->prof.free_events) (void)hipEventDestroy(e);
    delete t;
}

ara_status ara_table_bytes(const ara_tables* t, int64_t* bytes) {
    if (!t || !bytes) return fail(ARA_ERR_INVALID_ARG, "NULL argument");
    *bytes = t->bytes;
    return ARA_OK;
}

ara_status ara_cached_memory(int64_t* held_bytes, int64_t* idle_bytes) {
    int device = 0;
    HIP_TRY(hipGetDevice(&device), "hipGetDevice");
    int64_t held = 0, idle = 0;
    ara::cache_stats(device, &held, &idle);
    if (held_bytes) *held_bytes = held;
    if (idle_bytes) *idle_bytes = idle;
    return ARA_OK;
}

ara_status ara_release_cached_memory(int64_t* bytes_released) {
    int device = 0;
    HIP_TRY(hipGetDevice(&device), "hipGetDevice");
    const int64_t freed = ara::cache_release(device);
    if (bytes_released) *bytes_released = freed;
    return ARA_OK;
}

ara_status ara_layout_info_get(const ara_tables* t, ara_layout_info* info) {
    if (!t || !info) return fail(ARA_ERR_INVALID_ARG, "NULL argument");
    ara_layout_info v{};
    v.image_parts = t->parts.P;
    v.partitioned_ids = t->parts.length;
    v.partitioned_bytes = t->parts.bytes;
    v.stream_parts = t->stream.P;
    v.stream_group_trials = t->stream.G;
    v.stream_groups = t->stream.NG;
    v.stream_ids = t->stream.length;
    v.stream_bytes = t->stream.bytes;
    *info = v;
    return ARA_OK;
}

ara_status ara_kernel_stats(ara_tables* t, int32_t kernel, int64_t* launches, double* total_ms, int32_t reset) {
    if (!t || kernel < 0 || kernel > ARA_KERNEL_AGGREGATE) return fail(ARA_ERR_INVALID_ARG, "bad argument");
    DeviceScope ds(t->device);
    std::lock_guard<std::mutex> g(t->prof_mu);
    auto& ps = t->prof;
    for (auto& p : ps.pending) {
        HIP_TRY(hipEventSynchronize(p.stop), "event synchronize");
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p.start, p.stop), "event elapsed");
        ps.launches[p.kind] += 1;
        ps.total_ms[p.kind] += ms;
        ps.free_events.push_back(p.start);
        ps.free_events.push_back(p.stop);
    }
    ps.pending.clear();
    if (launches) *launches = ps.launches[kernel];
    if (total_ms) *total_ms = ps.total_ms[kernel];
    if (reset) {
        ps.launches[kernel] = 0;
        ps.total_ms[kernel] = 0.0;
    }
    return ARA_OK;
}

ara_status ara_set_tuning(ara_tables* t, const ara_tuning* tu) {
    if (!t) return fail(ARA_ERR_INVALID_ARG, "NULL tables");
    ara_tuning v{};
    if (tu) v = *tu;
    if (v.lanes_per_trial != 0 && v.lanes_per_trial != 8 && v.lanes_per_trial != 16 &&
        v.lanes_per_trial != 32 && v.lanes_per_trial != 64)
        return fail(ARA_ERR_INVALID_ARG, "lanes_per_trial must be 8, 16, 32 or 64");
    if (v.blocks_per_cu < 0 || v.blocks_per_cu > 64) return fail(ARA_ERR_INVALID_ARG, "blocks_per_cu in [0, 64]");
    if (v.part_lanes_per_trial != 0 && v.part_lanes_per_trial != 8 && v.part_lanes_per_trial != 16 &&
        v.part_lanes_per_trial != 32 && v.part_lanes_per_trial != 64)
        return fail(ARA_ERR_INVALID_ARG, "part_lanes_per_trial must be 8, 16, 32 or 64");
    if (v.schedule < 0 || v.schedule > 1) return fail(ARA_ERR_INVALID_ARG, "schedule must be 0 or 1");
    if (v.pass_variant < 0 || v.pass_variant > 2) return fail(ARA_ERR_INVALID_ARG, "pass_variant must be 0, 1 or 2");
    std::lock_guard<std::mutex> g(t->mu);
    t->tuning = v;
    return ARA_OK;
}

ara_status ara_get_tuning(const ara_tables* t, ara_tuning* tu) {
    if (!t || !tu) return fail(ARA_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(const_cast<ara_tables*>(t)->mu);
    *tu = t->tuning;
    return ARA_OK;
}

ara_status ara_footprint(const ara_tables* t, const ara_layer* layers, int32_t n_layers, uint32_t flags,
                         int64_t* bytes) {
    if (!t || !bytes || (n_layers > 0 && !layers) || n_layers < 0)
        return fail(ARA_ERR_INVALID_ARG, "NULL argument or negative layer count");
    int64_t total = 0;
    for (int i = 0; i < n_layers; ++i) total += layers[i].trial_count;
    int64_t b = 0;
    if (!(flags & ARA_LITERAL)) b += sizeof(double) * t->C;            // occurrence losses
    if (!(flags & ARA_LITERAL) && t->parts.P > 0) {
        int64_t most = 0;
        for (int i = 0; i < n_layers; ++i) most = std::max(most, layers[i].trial_count);
        ara_tuning tu;
        {
            std::lock_guard<std::mutex> g(const_cast<ara_tables*>(t)->mu);
            tu = t->tuning;
        }
        b += ara::part_scratch_bytes(t->C, t->parts.P) + static_cast<int64_t>(SplitPass(t, tu).partial_bytes(most));
    }
    if (!(flags & ARA_DEVICE_PTR)) b += sizeof(double) * total;       // staged output
    if (flags & (ARA_CHECKPOINT_S | ARA_CHECKPOINT_STRIDE)) b += 2 * sizeof(double) * total;
    if (flags & ARA_CHECKPOINT_STRIDE) b += sizeof(double) * (t->n_events / ara::kStride + 1);
    *bytes = b;
    return ARA_OK;
}

ara_status ara_yet_footprint(int64_t n_trials, int64_t n_events, int64_t catalogue_size, uint32_t flags,
                             int64_t* bytes) {
    if (!bytes || n_trials < 0 || n_events < 0 || catalogue_size < 1)
        return fail(ARA_ERR_INVALID_ARG, "NULL output or negative size");
    const int64_t N = n_trials, E = n_events;
    int64_t b = 8 * (N + 1) + 4 * (E + ara::kIdPad) + 64;          // offsets, IDs, validation flag
    int64_t temp = 0;
    if (!(flags & ARA_PLAIN_LAYOUT) && N > 0) {
        // 32-bit partitioned copy: IDs, segment padding (< 4 per segment,
        // < 32 per tile), segment starts, tile starts; counts while building
        const int64_t P = (catalogue_size + (int64_t(1) << ara::kImgShift) - 1) >> ara::kImgShift;
        if (P <= ara::kMaxParts) {
            const int64_t T = 256, tiles = (N + T - 1) / T;
            b += 4 * (E + 3 * N * P + 32 * tiles + ara::kIdPad) + 4 * tiles * (T * P + 1) + 8 * (tiles + 1);
            temp = std::max(temp, 4 * N * P + 8 * tiles);
        }
        // 16-bit copy: IDs (groups of at least 16 trials padded to 8 IDs per
        // part), trial ends and group starts, part bases; counts while building
        const int64_t Q = (catalogue_size + (int64_t(1) << ara::kStreamShift) - 1) >> ara::kStreamShift;
        if (Q <= ara::kMaxStreamParts) {
            const int64_t NG = (N + 15) / 16;
            b += 2 * (E + 7 * Q * NG + 512) + 2 * ara::kStreamGroupSlots * Q * NG + 4 * Q * (NG + 1) + 8 * (Q + 1);
            temp = std::max(temp, 4 * N * Q + 4 * Q * NG + 8 * Q + 4);
        }
    }
    *bytes = b + temp;
    return ARA_OK;
}

ara_status ara_metrics_footprint(int64_t n_trials, int32_t n_probs, uint32_t flags, int64_t* bytes) {
    if (!bytes || n_trials < 0 || n_probs < 0 || n_probs > 4) return fail(ARA_ERR_INVALID_ARG, "bad argument");
    int64_t b = ara::metrics_scratch_bytes(n_probs, n_trials);
    if (!(flags & ARA_DEVICE_PTR)) b += 8 * n_trials + 8 * (1 + 2 * static_cast<int64_t>(n_probs));
    *bytes = b;
    return ARA_OK;
}

ara_status ara_run_layers(ara_tables* t, const ara_layer* layers, int32_t n_layers, double* ylt,
                          int64_t ylt_capacity, uint32_t flags, void* stream) {
    if (!t || !layers || n_layers < 1) return fail(ARA_ERR_INVALID_ARG, "NULL argument or no layer");
    if (flags & ARA_CHECKPOINT_STRIDE) flags |= ARA_CHECKPOINT_S;
    const bool ckpt = (flags & ARA_CHECKPOINT_S) != 0;
    if (ckpt && n_layers != 1) return fail(ARA_ERR_UNSUPPORTED, "ARA_CHECKPOINT_S takes exactly one layer");
    std::vector<ara::LayerArgs> L(n_layers);
    int64_t total = 0;
    for (int i = 0; i < n_layers; ++i) {
        ara_status st = build_layer_args(t, layers[i], L[i]);
        if (st != ARA_OK) return st;
        L[i].out_offset = total;
        total += L[i].trial_count;
    }
    if (total == 0) return ARA_OK;
    if (!ylt) return fail(ARA_ERR_INVALID_ARG, "ylt is NULL");
    if (ylt_capacity < total)
        return fail(ARA_ERR_BUFFER_TOO_SMALL, "ylt holds %lld values, %lld needed", (long long)ylt_capacity,
                    (long long)total);
    DeviceScope ds(t->device);
    if (!ds.ok) return fail(ARA_ERR_DEVICE, "cannot select the tables' device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    UseFence use_fence(t, s);           // the tables' memory outlives this call's work
    const bool dev_out = (flags & ARA_DEVICE_PTR) != 0;
    const bool literal = (flags & ARA_LITERAL) != 0;
    ara_tuning tu;
    {
        std::lock_guard<std::mutex> g(t->mu);
        tu = t->tuning;
    }
    PoolBuffer staged;
    double* out = ylt;
    if (!dev_out) {
        HIP_TRY(staged.alloc(sizeof(double) * (total > 0 ? total : 1), s), "scratch for YLT");
        out = static_cast<double*>(staged.p);
    }
    // the partitioned passes serve plain runs.  Stride checkpoints need time
    // order: after the streaming or XCD-affine pass a time-ordered pass of their
    // own writes them; with pass_variant 1 the time-ordered trial pass does all
    const bool stride = (flags & ARA_CHECKPOINT_STRIDE) != 0;
    const bool use_parts = !literal && t->parts.P > 0 && !(stride && tu.pass_variant == 1);
    // the streaming pass (default) and the XCD-affine pass (pass_variant 2)
    // write per-part partial sums; pass_variant 1 selects the rank-based pass
    // with the compact value array
    const bool use_xcd = use_parts && tu.pass_variant != 1;
    const SplitPass split(t, tu);
    // several layers run as one persistent rank-based launch with pass_variant
    // 1; with the streaming (default) or XCD-affine pass they run one launch
    // sequence per layer, which ARA_GRAPH captures and replays as a whole
    const bool batched = n_layers > 1 && !(flags & ARA_PER_LAYER) && !literal && !ckpt && t->parts.P > 0 &&
                         tu.pass_variant == 1;
    const bool xgraph = (flags & ARA_GRAPH) && use_xcd && !ckpt;
    // one kept scratch buffer for the per-layer path: occurrence losses, part
    // images, partial sums (the batched path and graphs keep their own)
    auto up = [](size_t n) { return (n + 255) & ~size_t(255); };
    const size_t o_bytes = literal ? 0 : up(sizeof(double) * t->C);
    const size_t p_bytes = use_parts ? up(static_cast<size_t>(ara::part_scratch_bytes(t->C, t->parts.P))) : 0;
    size_t x_bytes = 0;
    if (use_xcd) {
        int64_t most = 0;
        for (int i = 0; i < n_layers; ++i) most = std::max(most, L[i].trial_count);
        x_bytes = up(split.partial_bytes(most));
    }
    ScratchLease lease(t->scratch_mu);
    lease.s = s;
    char* base = nullptr;
    if (!batched && !xgraph) {
        HIP_TRY(scratch_acquire(t->scratch_mu, t->scratch, o_bytes + p_bytes + x_bytes + 256, s, &lease.b),
                "scratch for occurrence losses, part images and partial sums");
        base = static_cast<char*>(lease.b->p);
    }
    struct {
        void* p;
    } obuf{base}, pbuf{base ? base + o_bytes : nullptr}, xbuf{base ? base + o_bytes + p_bytes : nullptr};
    double* S_buf = nullptr;
    double* stride_buf = nullptr;
    std::unique_lock<std::mutex> ck_lock(t->mu, std::defer_lock);
    if (ckpt) {
        ck_lock.lock();
        auto& ck = t->ck;
        ck.valid = false;
        if (ck.count < L[0].trial_count || !ck.S) {
            if (ck.S) (void)hipFree(ck.S);
            if (ck.ylt) (void)hipFree(ck.ylt);
            ck.S = ck.ylt = nullptr;
            const size_t nb = sizeof(double) * (L[0].trial_count > 0 ? L[0].trial_count : 1);
            HIP_TRY(hipMalloc(&ck.S, nb), "checkpoint S");
            HIP_TRY(hipMalloc(&ck.ylt, nb), "checkpoint YLT");
            ck.count = L[0].trial_count;
        }
        ck.has_stride = false;
        if (flags & ARA_CHECKPOINT_STRIDE) {
            if (!ck.stride) HIP_TRY(hipMalloc(&ck.stride, sizeof(double) * (t->n_events / ara::kStride + 1)),
                                    "stride checkpoints");
            HIP_TRY(ara::launch_fill(ck.stride, t->n_events / ara::kStride + 1, std::nan(""), s), "fill");
            stride_buf = ck.stride;
            ck.has_stride = true;
        }
        S_buf = ck.S;
    }
    if ((flags & ARA_GRAPH) && (batched || xgraph) && (!dev_out || s == nullptr))
        return fail(ARA_ERR_INVALID_ARG, "ARA_GRAPH needs a device output and a non-null stream");
    if (xgraph) {
        // key: the pass captured, layer count, output, trial ranges (terms and
        // ELT choices may change); -1: not a batched plan
        std::vector<int64_t> key{-1, split.stream ? 1 : 0, static_cast<int64_t>(n_layers),
                                 reinterpret_cast<int64_t>(out)};
        int64_t most = 0;
        for (int i = 0; i < n_layers; ++i) {
            key.push_back(L[i].trial_begin);
            key.push_back(L[i].trial_count);
            most = std::max(most, L[i].trial_count);
        }
        const size_t la_bytes = up(sizeof(ara::LayerArgs) * n_layers);
        const size_t xg_bytes = up(split.partial_bytes(most));
        const bool prof = (flags & ARA_PROFILE) != 0;
        std::lock_guard<std::mutex> g(t->stage_mu);
        ara::GraphEntry* ge = nullptr;
        for (auto* c : t->graphs)
            if (c->key == key) ge = c;
        auto upload = [&](ara::GraphEntry* e) -> hipError_t {
            return upload_layer_args(e, L.data(), sizeof(ara::LayerArgs) * n_layers, s);
        };
        if (!ge) {
            ge = new ara::GraphEntry();
            ge->key = key;
            hipError_t e = hipMalloc(&ge->scratch, la_bytes + o_bytes + p_bytes + xg_bytes);
            if (e != hipSuccess) {
                free_graph(ge);
                return hip_fail(e, "graph scratch");
            }
            char* gb = static_cast<char*>(ge->scratch);
            const ara::LayerArgs* dL = reinterpret_cast<const ara::LayerArgs*>(gb);
            double* go = reinterpret_cast<double*>(gb + la_bytes);
            void* gp = gb + la_bytes + o_bytes;
            void* gx = gb + la_bytes + o_bytes + p_bytes;
            if ((e = upload(ge)) != hipSuccess || (e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) !=
                                                      hipSuccess) {
                free_graph(ge);
                return hip_fail(e, "graph capture");
            }
            hipError_t le = hipSuccess;
            for (int i = 0; i < n_layers && le == hipSuccess; ++i) {
                le = ara::launch_fold_parts(t->sparse, t->C, L[i], dL + i, go, t->parts.P, gp, s);
                if (le == hipSuccess) le = split.pass(L[i], gp, gx, s);
                if (le == hipSuccess) le = split.combine(L[i], dL + i, gx, out + L[i].out_offset, nullptr, s);
            }
            e = hipStreamEndCapture(s, &ge->graph);
            if (le != hipSuccess || e != hipSuccess ||
                (e = hipGraphInstantiate(&ge->exec, ge->graph, nullptr, nullptr, 0)) != hipSuccess) {
                free_graph(ge);
                return hip_fail(le != hipSuccess ? le : e, "graph instantiate");
            }
            if (t->graphs.size() >= 8) {
                free_graph(t->graphs.front());
                t->graphs.erase(t->graphs.begin());
            }
            t->graphs.push_back(ge);
        } else {
            HIP_TRY(upload(ge), "upload layer terms");
        }
        KernelTimer kt(t, s, prof, ARA_KERNEL_BATCHED);
        HIP_TRY(hipGraphLaunch(ge->exec, s), "graph launch");
        kt.done();
        return ARA_OK;
    }
    if (batched) {
        BatchPlan plan = make_plan(t, L, out, tu.schedule);
        const int64_t n_items = static_cast<int64_t>(plan.items.size());
        const int64_t n_elts_total = static_cast<int64_t>(plan.idx.size());
        const int64_t sbytes = ara::batched_scratch_bytes(t->C, t->parts.P, n_layers, n_items, n_elts_total);
        const bool prof = (flags & ARA_PROFILE) != 0;
        if (flags & ARA_GRAPH) {
            std::lock_guard<std::mutex> g(t->stage_mu);
            ara::GraphEntry* ge = nullptr;
            for (auto* c : t->graphs)
                if (c->key == plan.key) ge = c;
            if (!ge) {
                ge = new ara::GraphEntry();
                ge->key = plan.key;
                hipError_t e = hipMalloc(&ge->scratch, sbytes);
                if (e != hipSuccess) {
                    free_graph(ge);
                    return hip_fail(e, "graph scratch");
                }
                ara::BatchedScratch bs =
                    ara::carve_batched(ge->scratch, t->C, t->parts.P, n_layers, n_items, n_elts_total);
                if ((e = upload_plan(ge->stage, plan, bs, true, s)) != hipSuccess ||
                    (e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
                    free_graph(ge);
                    return hip_fail(e, "graph capture");
                }
                hipError_t le = ara::launch_batched(t->parts, t->n_trials, t->C, t->elts, n_layers, bs, n_items, out,
                                                    t->n_cu, s, nullptr, nullptr, tu.part_lanes_per_trial);
                e = hipStreamEndCapture(s, &ge->graph);
                if (le != hipSuccess || e != hipSuccess ||
                    (e = hipGraphInstantiate(&ge->exec, ge->graph, nullptr, nullptr, 0)) != hipSuccess) {
                    free_graph(ge);
                    return hip_fail(le != hipSuccess ? le : e, "graph instantiate");
                }
                if (t->graphs.size() >= 8) {
                    free_graph(t->graphs.front());
                    t->graphs.erase(t->graphs.begin());
                }
                t->graphs.push_back(ge);
            } else {
                ara::BatchedScratch bs =
                    ara::carve_batched(ge->scratch, t->C, t->parts.P, n_layers, n_items, n_elts_total);
                HIP_TRY(upload_plan(ge->stage, plan, bs, false, s), "upload layer terms");
            }
            KernelTimer kt(t, s, prof, ARA_KERNEL_BATCHED);
            HIP_TRY(hipGraphLaunch(ge->exec, s), "graph launch");
            kt.done();
        } else {
            PoolBuffer bbuf;
            HIP_TRY(bbuf.alloc(sbytes, s), "batched scratch");
            ara::BatchedScratch bs = ara::carve_batched(bbuf.p, t->C, t->parts.P, n_layers, n_items, n_elts_total);
            {
                std::lock_guard<std::mutex> g(t->stage_mu);
                HIP_TRY(upload_plan(t->stage, plan, bs, true, s), "upload work list");
            }
            KernelTimer kt(t, s, prof, ARA_KERNEL_BATCHED);
            HIP_TRY(ara::launch_batched(t->parts, t->n_trials, t->C, t->elts, n_layers, bs, n_items, out, t->n_cu, s,
                                        nullptr, nullptr, tu.part_lanes_per_trial),
                    "batched pass");
            kt.done();
        }
    }
    for (int i = 0; i < n_layers && !batched; ++i) {
        ara::TrialPassArgs a{};
        a.offsets = t->offsets;
        a.ids = t->ids;
        a.elts = t->elts;
        a.C = t->C;
        a.o = static_cast<const double*>(obuf.p);
        a.ylt = out + L[i].out_offset;
        a.S = S_buf;
        a.stride = stride_buf;
        const bool prof = (flags & ARA_PROFILE) != 0;
        if (!literal) {
            KernelTimer kt(t, s, prof, ARA_KERNEL_FOLD);
            if (use_parts)
                HIP_TRY(ara::launch_fold_parts(t->sparse, t->C, L[i], nullptr, static_cast<double*>(obuf.p), t->parts.P,
                                               pbuf.p, s),
                        "fold and part images");
            else
                HIP_TRY(ara::launch_fold(t->elts, t->C, L[i], static_cast<double*>(obuf.p), tu, s), "fold");
            kt.done();
        }
        if (use_xcd) {
            KernelTimer kp(t, s, prof, ARA_KERNEL_TRIAL_PASS);
            HIP_TRY(split.pass(L[i], pbuf.p, xbuf.p, s), "trial pass");
            kp.done();
            KernelTimer kc(t, s, prof, ARA_KERNEL_COMBINE);
            HIP_TRY(split.combine(L[i], nullptr, xbuf.p, a.ylt, a.S, s), "partial sums merge");
            kc.done();
            if (stride_buf) {
                PoolBuffer probe;
                HIP_TRY(probe.alloc(static_cast<size_t>(ara::probe_table_bytes(t->C)), s), "scratch for probe words");
                HIP_TRY(ara::launch_stride_checkpoints(t->offsets, t->ids, pbuf.p, t->parts.P, t->C,
                                                       static_cast<uint64_t*>(probe.p), L[i], stride_buf, t->n_cu, s),
                        "stride checkpoints");
            }
            continue;
        }
        KernelTimer kt(t, s, prof, ARA_KERNEL_TRIAL_PASS);
        if (use_parts)
            HIP_TRY(ara::launch_part_pass(t->parts, t->n_trials, L[i], pbuf.p, a.ylt, a.S, t->n_cu, s,
                                          tu.part_lanes_per_trial),
                    "partitioned trial pass");
        else
            HIP_TRY(ara::launch_trial_pass(a, L[i], literal, tu, t->n_cu, s), "trial pass");
        kt.done();
    }
    if (ckpt) {
        HIP_TRY(hipMemcpyAsync(t->ck.ylt, out, sizeof(double) * L[0].trial_count, hipMemcpyDeviceToDevice, s),
                "keep YLT");
        t->ck.key = L[0];
        t->ck.valid = true;
    }
    if (!dev_out) {
        HIP_TRY(hipMemcpyAsync(ylt, out, sizeof(double) * total, hipMemcpyDeviceToHost, s), "copy YLT");
        HIP_TRY(hipStreamSynchronize(s), "synchronize");
    }
    return ARA_OK;
}

ara_status ara_run_portfolio(ara_tables* t, const ara_program* programs, int32_t n_programs, int32_t n_splits,
                             const ara_portfolio_out* out, uint32_t flags, void* stream) {
    if (!t || !programs || !out) return fail(ARA_ERR_INVALID_ARG, "NULL argument");
    if (n_programs < 1) return fail(ARA_ERR_INVALID_ARG, "a portfolio needs at least one program");
    if (n_programs > ARA_MAX_PROGRAMS)
        return fail(ARA_ERR_UNSUPPORTED, "%d programs, at most %d", n_programs, ARA_MAX_PROGRAMS);
    if (n_splits < 1) return fail(ARA_ERR_INVALID_ARG, "n_splits must be >= 1");
    if (!out->layer_ylt && !out->program_ylt && !out->portfolio_ylt) return fail(ARA_ERR_INVALID_ARG, "no output");
    if (flags & (ARA_CHECKPOINT_S | ARA_CHECKPOINT_STRIDE | ARA_GRAPH))
        return fail(ARA_ERR_INVALID_ARG, "ara_run_portfolio takes ARA_DEVICE_PTR, ARA_LITERAL and ARA_PROFILE");
    std::vector<ara::LayerArgs> L;
    ara::PortfolioSumArgs agg{};
    agg.n_programs = n_programs;
    agg.first[0] = 0;
    for (int p = 0; p < n_programs; ++p) {
        if (programs[p].n_layers < 1 || !programs[p].layers)
            return fail(ARA_ERR_INVALID_ARG, "program %d has no layers", p);
        for (int i = 0; i < programs[p].n_layers; ++i) {
            ara::LayerArgs a;
            ara_status st = build_layer_args(t, programs[p].layers[i], a);
            if (st != ARA_OK) return st;
            if (!L.empty() && (a.trial_begin != L[0].trial_begin || a.trial_count != L[0].trial_count))
                return fail(ARA_ERR_INVALID_ARG, "program %d layer %d covers other trials than the first layer", p, i);
            L.push_back(a);
        }
        agg.first[p + 1] = static_cast<int32_t>(L.size());
    }
    const int64_t n_layers = static_cast<int64_t>(L.size());
    const int64_t begin = L[0].trial_begin, n = L[0].trial_count;
    if (out->layer_ylt && out->layer_capacity < n_layers * n)
        return fail(ARA_ERR_BUFFER_TOO_SMALL, "layer_ylt holds %lld values, %lld needed",
                    (long long)out->layer_capacity, (long long)(n_layers * n));
    if (out->program_ylt && out->program_capacity < n_programs * n)
        return fail(ARA_ERR_BUFFER_TOO_SMALL, "program_ylt holds %lld values, %lld needed",
                    (long long)out->program_capacity, (long long)(n_programs * n));
    if (out->portfolio_ylt && out->portfolio_capacity < n)
        return fail(ARA_ERR_BUFFER_TOO_SMALL, "portfolio_ylt holds %lld values, %lld needed",
                    (long long)out->portfolio_capacity, (long long)n);
    if (n == 0) return ARA_OK;
    DeviceScope ds(t->device);
    if (!ds.ok) return fail(ARA_ERR_DEVICE, "cannot select the tables' device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    UseFence use_fence(t, s);           // the tables' memory outlives this call's work
    const bool dev_out = (flags & ARA_DEVICE_PTR) != 0;
    const bool literal = (flags & ARA_LITERAL) != 0;
    const bool prof = (flags & ARA_PROFILE) != 0;
    ara_tuning tu;
    {
        std::lock_guard<std::mutex> g(t->mu);
        tu = t->tuning;
    }
    const bool use_parts = !literal && t->parts.P > 0;
    const bool use_xcd = use_parts && tu.pass_variant != 1;
    const SplitPass split(t, tu);
    // split i covers [b(i), b(i + 1)): Algorithm 1's YET_i
    auto split_at = [&](int64_t i) { return begin + (n * i) / n_splits; };
    int64_t most = 0;
    for (int64_t i = 0; i < n_splits; ++i) most = std::max(most, split_at(i + 1) - split_at(i));
    // one kept scratch buffer: occurrence losses, part images, partial sums of
    // the largest split, and whatever output the caller keeps on the host
    auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
    const size_t o_bytes = literal ? 0 : up(sizeof(double) * t->C);
    const size_t p_bytes = use_parts ? up(static_cast<size_t>(ara::part_scratch_bytes(t->C, t->parts.P))) : 0;
    const size_t x_bytes = use_xcd ? up(split.partial_bytes(most)) : 0;
    const bool stage_layers = !dev_out || !out->layer_ylt;
    const size_t l_bytes = stage_layers ? up(sizeof(double) * n_layers * n) : 0;
    const size_t g_bytes = !dev_out && out->program_ylt ? up(sizeof(double) * n_programs * n) : 0;
    const size_t f_bytes = !dev_out && out->portfolio_ylt ? up(sizeof(double) * n) : 0;
    ScratchLease lease(t->scratch_mu);
    lease.s = s;
    HIP_TRY(scratch_acquire(t->scratch_mu, t->scratch, o_bytes + p_bytes + x_bytes + l_bytes + g_bytes + f_bytes + 256,
                            s, &lease.b),
            "portfolio scratch");
    char* base = static_cast<char*>(lease.b->p);
    double* o_buf = reinterpret_cast<double*>(base);
    void* p_buf = base + o_bytes;
    void* x_buf = base + o_bytes + p_bytes;
    double* layer_rows = stage_layers ? reinterpret_cast<double*>(base + o_bytes + p_bytes + x_bytes) : out->layer_ylt;
    double* program_rows = nullptr;
    double* portfolio_row = nullptr;
    if (out->program_ylt)
        program_rows = dev_out ? out->program_ylt
                               : reinterpret_cast<double*>(base + o_bytes + p_bytes + x_bytes + l_bytes);
    if (out->portfolio_ylt)
        portfolio_row = dev_out ? out->portfolio_ylt
                                : reinterpret_cast<double*>(base + o_bytes + p_bytes + x_bytes + l_bytes + g_bytes);
    for (int64_t l = 0; l < n_layers; ++l) {
        if (!literal) {
            KernelTimer kt(t, s, prof, ARA_KERNEL_FOLD);
            if (use_parts)
                HIP_TRY(ara::launch_fold_parts(t->sparse, t->C, L[l], nullptr, o_buf, t->parts.P, p_buf, s),
                        "fold and part images");
            else
                HIP_TRY(ara::launch_fold(t->elts, t->C, L[l], o_buf, tu, s), "fold");
            kt.done();
        }
        for (int64_t i = 0; i < n_splits; ++i) {
            ara::LayerArgs Li = L[l];
            Li.trial_begin = split_at(i);
            Li.trial_count = split_at(i + 1) - Li.trial_begin;
            if (Li.trial_count == 0) continue;
            double* ylt_i = layer_rows + l * n + (Li.trial_begin - begin);
            if (use_xcd) {
                KernelTimer kp(t, s, prof, ARA_KERNEL_TRIAL_PASS);
                HIP_TRY(split.pass(Li, p_buf, x_buf, s), "trial pass");
                kp.done();
                KernelTimer kc(t, s, prof, ARA_KERNEL_COMBINE);
                HIP_TRY(split.combine(Li, nullptr, x_buf, ylt_i, nullptr, s), "partial sums merge");
                kc.done();
            } else if (use_parts) {
                KernelTimer kp(t, s, prof, ARA_KERNEL_TRIAL_PASS);
                HIP_TRY(ara::launch_part_pass(t->parts, t->n_trials, Li, p_buf, ylt_i, nullptr, t->n_cu, s,
                                              tu.part_lanes_per_trial),
                        "partitioned trial pass");
                kp.done();
            } else {
                ara::TrialPassArgs a{};
                a.offsets = t->offsets;
                a.ids = t->ids;
                a.elts = t->elts;
                a.C = t->C;
                a.o = o_buf;
                a.ylt = ylt_i;
                KernelTimer kp(t, s, prof, ARA_KERNEL_TRIAL_PASS);
                HIP_TRY(ara::launch_trial_pass(a, Li, literal, tu, t->n_cu, s), "trial pass");
                kp.done();
            }
        }
    }
    if (program_rows || portfolio_row) {
        agg.layer_ylt = layer_rows;
        agg.count = n;
        agg.program_ylt = program_rows;
        agg.portfolio_ylt = portfolio_row;
        KernelTimer ka(t, s, prof, ARA_KERNEL_AGGREGATE);
        HIP_TRY(ara::launch_portfolio_sum(agg, t->n_cu, s), "program and portfolio sums");
        ka.done();
    }
    if (!dev_out) {
        if (out->layer_ylt)
            HIP_TRY(hipMemcpyAsync(out->layer_ylt, layer_rows, sizeof(double) * n_layers * n, hipMemcpyDeviceToHost, s),
                    "copy layer YLTs");
        if (out->program_ylt)
            HIP_TRY(hipMemcpyAsync(out->program_ylt, program_rows, sizeof(double) * n_programs * n,
                                   hipMemcpyDeviceToHost, s),
                    "copy program YLTs");
        if (out->portfolio_ylt)
            HIP_TRY(hipMemcpyAsync(out->portfolio_ylt, portfolio_row, sizeof(double) * n, hipMemcpyDeviceToHost, s),
                    "copy portfolio YLT");
        HIP_TRY(hipStreamSynchronize(s), "synchronize");
    }
    return ARA_OK;
}

ara_status ara_risk_metrics(const double* ylt, int64_t n_trials, const double* probs, int32_t n_probs,
                            double* mean_out, double* pml_out, double* tvar_out, uint32_t flags, void* stream) {
    if (!ylt || !mean_out || n_probs < 0 || (n_probs > 0 && (!probs || !pml_out || !tvar_out)))
        return fail(ARA_ERR_INVALID_ARG, "NULL argument");
    if (n_trials < 1) return fail(ARA_ERR_INVALID_ARG, "need at least one trial");
    if (n_probs > 4) return fail(ARA_ERR_UNSUPPORTED, "at most 4 probabilities per call");
    std::vector<int64_t> m(n_probs);
    for (int q = 0; q < n_probs; ++q) {
        if (!(probs[q] > 0.0 && probs[q] < 1.0)) return fail(ARA_ERR_INVALID_ARG, "p must lie in (0, 1)");
        m[q] = tail_count(n_trials, probs[q]);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    int device = 0;
    HIP_TRY(hipGetDevice(&device), "hipGetDevice");
    const int n_cu = query_cu_count(device);
    const bool dev = (flags & ARA_DEVICE_PTR) != 0;
    PoolBuffer staged_in, results;
    // kept per device, like the tables' scratch (see ScratchBuffer)
    static std::mutex metrics_mu;
    static std::list<std::pair<int, std::vector<ara::ScratchBuffer*>>> metrics_sets;   // stable addresses
    std::vector<ara::ScratchBuffer*>* sets = nullptr;
    {
        std::lock_guard<std::mutex> g(metrics_mu);
        for (auto& d : metrics_sets)
            if (d.first == device) sets = &d.second;
        if (!sets) {
            metrics_sets.emplace_back(device, std::vector<ara::ScratchBuffer*>());
            sets = &metrics_sets.back().second;
        }
    }
    ScratchLease scratch(metrics_mu);
    scratch.s = s;
    HIP_TRY(scratch_acquire(metrics_mu, *sets, static_cast<size_t>(ara::metrics_scratch_bytes(n_probs, n_trials)), s,
                            &scratch.b),
            "metrics scratch");
    if (!dev) HIP_TRY(results.alloc(sizeof(double) * (1 + 2 * n_probs), s), "metrics results");
    const double* x = ylt;
    if (!dev) {
        HIP_TRY(staged_in.alloc(sizeof(double) * n_trials, s), "metrics input");
        HIP_TRY(hipMemcpyAsync(staged_in.p, ylt, sizeof(double) * n_trials, hipMemcpyHostToDevice, s), "copy YLT");
        x = static_cast<const double*>(staged_in.p);
    }
    double* r = static_cast<double*>(results.p);
    // device outputs are written by the kernels themselves; host outputs go
    // through the results buffer [mean, PML_0, TVaR_0, PML_1, ...]
    const ara::MetricsOut out = dev ? ara::MetricsOut{mean_out, pml_out, tvar_out, 1}
                                    : ara::MetricsOut{r, r + 1, r + 2, 2};
    // the scratch counts as primed only once this whole sequence is enqueued
    const bool primed = scratch.b->primed;
    scratch.b->primed = false;
    HIP_TRY(ara::launch_metrics(x, n_trials, m.data(), n_probs, scratch.b->p, primed, out, n_cu, s), "metrics kernels");
    scratch.b->primed = true;
    if (dev) return ARA_OK;
    std::vector<double> h(1 + 2 * n_probs);
    HIP_TRY(hipMemcpyAsync(h.data(), r, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s), "copy metrics");
    HIP_TRY(hipStreamSynchronize(s), "synchronize");
    if (std::isnan(h[0])) return fail(ARA_ERR_INVALID_ARG, "year losses must be >= 0 and not NaN");
    *mean_out = h[0];
    for (int q = 0; q < n_probs; ++q) {
        pml_out[q] = h[1 + 2 * q];
        tvar_out[q] = h[2 + 2 * q];
    }
    return ARA_OK;
}

ara_status ara_analyze(ara_tables* t, const ara_layer* layer, const double* probs, int32_t n_probs, double* ylt,
                       int64_t ylt_capacity, double* metrics, uint32_t flags, void* stream) {
    if (!t || !layer || !ylt || !metrics || n_probs < 0 || (n_probs > 0 && !probs))
        return fail(ARA_ERR_INVALID_ARG, "NULL argument");
    if (n_probs > 4) return fail(ARA_ERR_UNSUPPORTED, "at most 4 probabilities per call");
    if (flags & ~static_cast<uint32_t>(ARA_DEVICE_PTR | ARA_GRAPH | ARA_PROFILE))
        return fail(ARA_ERR_INVALID_ARG, "flags: ARA_DEVICE_PTR, ARA_GRAPH and ARA_PROFILE only");
    ara::LayerArgs L;
    ara_status st = build_layer_args(t, *layer, L);
    if (st != ARA_OK) return st;
    if (L.trial_count < 1) return fail(ARA_ERR_INVALID_ARG, "layer has no trials");
    if (ylt_capacity < L.trial_count)
        return fail(ARA_ERR_BUFFER_TOO_SMALL, "ylt holds %lld values, %lld needed", (long long)ylt_capacity,
                    (long long)L.trial_count);
    std::vector<int64_t> m(n_probs);
    for (int q = 0; q < n_probs; ++q) {
        if (!(probs[q] > 0.0 && probs[q] < 1.0)) return fail(ARA_ERR_INVALID_ARG, "p must lie in (0, 1)");
        m[q] = tail_count(L.trial_count, probs[q]);
    }
    const bool dev = (flags & ARA_DEVICE_PTR) != 0;
    if ((flags & ARA_GRAPH) && (!dev || !stream))
        return fail(ARA_ERR_INVALID_ARG, "ARA_GRAPH needs device outputs and a non-null stream");
    ara_tuning tu;
    {
        std::lock_guard<std::mutex> g(t->mu);
        tu = t->tuning;
    }
    if (!(flags & ARA_GRAPH) || t->parts.P <= 0 || tu.pass_variant == 1) {
        // the two calls one after the other (as ara_run_layers, no graph for
        // the plain layout or the rank-based pass of pass_variant 1)
        st = ara_run_layers(t, layer, 1, ylt, ylt_capacity, flags & (ARA_DEVICE_PTR | ARA_PROFILE), stream);
        if (st != ARA_OK) return st;
        return ara_risk_metrics(ylt, L.trial_count, probs, n_probs, metrics, metrics + 1, metrics + 1 + n_probs,
                                flags & ARA_DEVICE_PTR, stream);
    }
    // one graph: fold, pass, combine and the metrics kernels, on scratch the
    // graph owns (the metrics part primed once; each replay leaves it ready
    // for the next).  Terms and ELT choices are read from device memory, so
    // new terms reuse the graph.
    DeviceScope ds(t->device);
    if (!ds.ok) return fail(ARA_ERR_DEVICE, "cannot select the tables' device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    UseFence use_fence(t, s);           // the tables' memory outlives this call's work
    const SplitPass split(t, tu);
    auto up = [](size_t n) { return (n + 255) & ~size_t(255); };
    const size_t la_bytes = up(sizeof(ara::LayerArgs));
    const size_t o_bytes = up(sizeof(double) * t->C);
    const size_t p_bytes = up(static_cast<size_t>(ara::part_scratch_bytes(t->C, t->parts.P)));
    const size_t xg_bytes = up(split.partial_bytes(L.trial_count));
    const size_t m_bytes = up(static_cast<size_t>(ara::metrics_scratch_bytes(n_probs, L.trial_count)));
    // what the graph bakes in: the outputs, the trial range, the pass and the tail counts
    std::vector<int64_t> key{-2, reinterpret_cast<int64_t>(ylt), reinterpret_cast<int64_t>(metrics), L.trial_begin,
                             L.trial_count, split.stream ? 1 : 0, n_probs};
    for (int q = 0; q < n_probs; ++q) key.push_back(m[q]);
    const bool prof = (flags & ARA_PROFILE) != 0;
    std::lock_guard<std::mutex> g(t->stage_mu);
    ara::GraphEntry* ge = nullptr;
    for (auto* c : t->graphs)
        if (c->key == key) ge = c;
    auto upload = [&](ara::GraphEntry* e) -> hipError_t { return upload_layer_args(e, &L, sizeof(L), s); };
    if (!ge) {
        ge = new ara::GraphEntry();
        ge->key = key;
        hipError_t e = hipMalloc(&ge->scratch, la_bytes + o_bytes + p_bytes + xg_bytes + m_bytes);
        if (e != hipSuccess) {
            free_graph(ge);
            return hip_fail(e, "graph scratch");
        }
        char* gb = static_cast<char*>(ge->scratch);
        const ara::LayerArgs* dL = reinterpret_cast<const ara::LayerArgs*>(gb);
        double* go = reinterpret_cast<double*>(gb + la_bytes);
        void* gp = gb + la_bytes + o_bytes;
        void* gx = gb + la_bytes + o_bytes + p_bytes;
        void* gm = gb + la_bytes + o_bytes + p_bytes + xg_bytes;
        if ((e = upload(ge)) != hipSuccess || (e = ara::launch_metrics_prime(gm, m.data(), n_probs, s)) != hipSuccess ||
            (e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
            free_graph(ge);
            return hip_fail(e, "graph capture");
        }
        hipError_t le = ara::launch_fold_parts(t->sparse, t->C, L, dL, go, t->parts.P, gp, s);
        if (le == hipSuccess) le = split.pass(L, gp, gx, s);
        if (le == hipSuccess) le = split.combine(L, dL, gx, ylt, nullptr, s);
        if (le == hipSuccess)
            le = ara::launch_metrics(ylt, L.trial_count, m.data(), n_probs, gm, true,
                                     ara::MetricsOut{metrics, metrics + 1, metrics + 1 + n_probs, 1}, t->n_cu, s);
        e = hipStreamEndCapture(s, &ge->graph);
        if (le != hipSuccess || e != hipSuccess ||
            (e = hipGraphInstantiate(&ge->exec, ge->graph, nullptr, nullptr, 0)) != hipSuccess) {
            free_graph(ge);
            return hip_fail(le != hipSuccess ? le : e, "graph instantiate");
        }
        if (t->graphs.size() >= 8) {
            free_graph(t->graphs.front());
            t->graphs.erase(t->graphs.begin());
        }
        t->graphs.push_back(ge);
    } else {
        HIP_TRY(upload(ge), "upload layer terms");
    }
    KernelTimer kt(t, s, prof, ARA_KERNEL_BATCHED);
    HIP_TRY(hipGraphLaunch(ge->exec, s), "graph launch");
    kt.done();
    return ARA_OK;
}

ara_status ara_risk_metrics_noalloc(const double* ylt, int64_t n_trials, const double* probs, int32_t n_probs,
                                    double* mean_out, double* pml_out, double* tvar_out, void* stream) {
    if (!ylt || !mean_out || n_probs < 0 || (n_probs > 0 && (!probs || !pml_out || !tvar_out)))
        return fail(ARA_ERR_INVALID_ARG, "NULL argument");
    if (n_trials < 1) return fail(ARA_ERR_INVALID_ARG, "need at least one trial");
    if (n_probs > 4) return fail(ARA_ERR_UNSUPPORTED, "at most 4 probabilities per call");
    int64_t m[4] = {0, 0, 0, 0};
    for (int q = 0; q < n_probs; ++q) {
        if (!(probs[q] > 0.0 && probs[q] < 1.0)) return fail(ARA_ERR_INVALID_ARG, "p must lie in (0, 1)");
        m[q] = tail_count(n_trials, probs[q]);
    }
    void* scratch = nullptr;
    int64_t capacity = 0;
    HIP_TRY(ara::metrics_noalloc_scratch(&scratch, &capacity), "static metrics scratch");
    const int64_t need = ara::metrics_scratch_bytes(n_probs, n_trials);
    if (need > capacity)
        return fail(ARA_ERR_UNSUPPORTED,
                    "%lld trials x %d probabilities need %lld bytes of scratch; the static scratch holds %lld "
                    "(n_probs * n_trials <= %lld); use ara_risk_metrics",
                    (long long)n_trials, n_probs, (long long)need, (long long)capacity,
                    (long long)ARA_METRICS_NOALLOC_KEYS);
    int device = 0;
    HIP_TRY(hipGetDevice(&device), "hipGetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // not primed: the first kernel clears the histograms, counters and flag
    // that earlier calls on this device left in the shared array
    HIP_TRY(ara::launch_metrics(ylt, n_trials, m, n_probs, scratch, false,
                                ara::MetricsOut{mean_out, pml_out, tvar_out, 1}, query_cu_count(device), s),
            "metrics kernels");
    return ARA_OK;
}

ara_status ara_backward(ara_tables* t, const ara_layer* layer, double tvar_p, double* grad_mean,
                        double* grad_tvar, uint32_t flags, void* stream) {
    if (!t || !layer) return fail(ARA_ERR_INVALID_ARG, "NULL argument");
    if (!(tvar_p > 0.0 && tvar_p < 1.0)) return fail(ARA_ERR_INVALID_ARG, "tvar_p must lie in (0, 1)");
    ara::LayerArgs L;
    ara_status st = build_layer_args(t, *layer, L);
    if (st != ARA_OK) return st;
    if (L.trial_count < 1) return fail(ARA_ERR_INVALID_ARG, "layer has no trials");
    std::lock_guard<std::mutex> g(t->mu);
    if (!t->ck.valid || !same_layer(t->ck.key, L))
        return fail(ARA_ERR_NOT_READY, "no checkpointed forward for this layer (run with ARA_CHECKPOINT_S)");
    DeviceScope ds(t->device);
    if (!ds.ok) return fail(ARA_ERR_DEVICE, "cannot select the tables' device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    UseFence use_fence(t, s);           // the tables' memory outlives this call's work
    const int P = 2 * L.J + 4;
    const bool dev = (flags & ARA_DEVICE_PTR) != 0;
    PoolBuffer scratch, staged;
    HIP_TRY(scratch.alloc(ara::adjoint_scratch_bytes(t->C, L.J, L.trial_count), s), "adjoint scratch");
    double* gm = grad_mean;
    double* gt = grad_tvar;
    if (!dev) {
        HIP_TRY(staged.alloc(sizeof(double) * 2 * P, s), "adjoint output");
        gm = grad_mean ? static_cast<double*>(staged.p) : nullptr;
        gt = grad_tvar ? static_cast<double*>(staged.p) + P : nullptr;
    }
    const int64_t m = tail_count(L.trial_count, tvar_p);
    // with the partitioned layout the histogram pass reads the nonzero bitmap
    // of the part images, rebuilt here from a fold of the layer
    PoolBuffer obuf, pbuf;
    const bool use_parts = t->parts.P > 0;
    // pass_variant 0: the histogram streams the 16-bit copy when the tables
    // hold one; else the XCD-affine pass over the 32-bit partitioned copy
    const bool use_stream = use_parts && t->tuning.pass_variant == 0 && t->stream.P > 0;
    if (use_parts) {
        const ara_tuning tu = t->tuning;   // t->mu is held
        HIP_TRY(obuf.alloc(sizeof(double) * t->C, s), "scratch for occurrence losses");
        HIP_TRY(pbuf.alloc(ara::part_scratch_bytes(t->C, t->parts.P), s), "scratch for part images");
        if (t->sparse.chunk_off) {
            // the forward's fold from the sparse pool (o, images and superblock counts)
            HIP_TRY(ara::launch_fold_parts(t->sparse, t->C, L, nullptr, static_cast<double*>(obuf.p), t->parts.P,
                                           pbuf.p, s),
                    "fold");
        } else {
            HIP_TRY(ara::launch_fold(t->elts, t->C, L, static_cast<double*>(obuf.p), tu, s), "fold");
            HIP_TRY(ara::launch_part_fold(static_cast<const double*>(obuf.p), t->C, t->parts.P, pbuf.p, s, false),
                    "images");
        }
    }
    HIP_TRY(ara::launch_adjoint(t->offsets, t->ids, t->elts, t->C, L, t->ck.S, t->ck.ylt, m, scratch.p, gm, gt,
                                t->n_cu, s, use_parts ? &t->parts : nullptr, pbuf.p, t->n_trials,
                                t->sparse.chunk_off ? &t->sparse : nullptr, use_stream ? &t->stream : nullptr),
            "adjoint kernels");
    if (!dev) {
        std::vector<double> h(2 * P);
        HIP_TRY(hipMemcpyAsync(h.data(), staged.p, sizeof(double) * 2 * P, hipMemcpyDeviceToHost, s), "copy");
        HIP_TRY(hipStreamSynchronize(s), "synchronize");
        if (grad_mean) std::memcpy(grad_mean, h.data(), sizeof(double) * P);
        if (grad_tvar) std::memcpy(grad_tvar, h.data() + P, sizeof(double) * P);
    }
    return ARA_OK;
}

ara_status ara_debug_lookups(ara_tables* t, const ara_layer* layer, int64_t trial, uint32_t* ids_out,
                             double* losses_out, int64_t capacity, int64_t* n_out, void* stream) {
    if (!t || !layer || !n_out || capacity < 0) return fail(ARA_ERR_INVALID_ARG, "NULL argument");
    if (trial < 0 || trial >= t->n_trials) return fail(ARA_ERR_INVALID_ARG, "trial outside the YET");
    ara_layer probe = *layer;
    probe.trial_begin = 0;
    probe.trial_count = 0;
    ara::LayerArgs L;
    ara_status st = build_layer_args(t, probe, L);
    if (st != ARA_OK) return st;
    DeviceScope ds(t->device);
    if (!ds.ok) return fail(ARA_ERR_DEVICE, "cannot select the tables' device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    UseFence use_fence(t, s);           // the tables' memory outlives this call's work
    int64_t be[2];
    HIP_TRY(hipMemcpyAsync(be, t->offsets + trial, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s), "offsets");
    HIP_TRY(hipStreamSynchronize(s), "synchronize");
    const int64_t K = be[1] - be[0];
    *n_out = K;
    if (K > capacity) return fail(ARA_ERR_BUFFER_TOO_SMALL, "trial has %lld events, capacity %lld",
                                  (long long)K, (long long)capacity);
    if (K == 0) return ARA_OK;
    if (!ids_out || (L.J > 0 && !losses_out)) return fail(ARA_ERR_INVALID_ARG, "NULL output");
    PoolBuffer dids, dloss;
    HIP_TRY(dids.alloc(sizeof(uint32_t) * K, s), "scratch");
    HIP_TRY(dloss.alloc(sizeof(double) * K * (L.J > 0 ? L.J : 1), s), "scratch");
    HIP_TRY(ara::launch_debug_lookups(t->offsets, t->ids, t->elts, t->C, L, trial, static_cast<uint32_t*>(dids.p),
                                      static_cast<double*>(dloss.p), s),
            "lookup kernel");
    HIP_TRY(hipMemcpyAsync(ids_out, dids.p, sizeof(uint32_t) * K, hipMemcpyDeviceToHost, s), "copy ids");
    if (L.J > 0)
        HIP_TRY(hipMemcpyAsync(losses_out, dloss.p, sizeof(double) * K * L.J, hipMemcpyDeviceToHost, s), "copy");
    HIP_TRY(hipStreamSynchronize(s), "synchronize");
    return ARA_OK;
}

ara_status ara_debug_read(ara_tables* t, const ara_layer* layer, int32_t what, void* out, int64_t capacity,
                          int64_t* n_out, void* stream) {
    if (!t || !n_out || capacity < 0) return fail(ARA_ERR_INVALID_ARG, "NULL argument");
    if (what < ARA_DEBUG_OCCURRENCE || what > ARA_DEBUG_STREAM_GEND) return fail(ARA_ERR_INVALID_ARG, "bad `what`");
    DeviceScope ds(t->device);
    if (!ds.ok) return fail(ARA_ERR_DEVICE, "cannot select the tables' device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    UseFence use_fence(t, s);           // the tables' memory outlives this call's work
    const void* src = nullptr;
    int64_t bytes = 0;
    PoolBuffer buf;
    if (what >= ARA_DEBUG_STREAM_IDS) {
        const ara::StreamLayout& st = t->stream;
        if (st.P == 0) return fail(ARA_ERR_UNSUPPORTED, "the tables hold no 16-bit stream copy");
        switch (what) {
            case ARA_DEBUG_STREAM_IDS: src = st.ids; bytes = sizeof(uint16_t) * st.length; break;
            case ARA_DEBUG_STREAM_BASE: src = st.part_base; bytes = sizeof(int64_t) * (st.P + 1); break;
            case ARA_DEBUG_STREAM_GSTART: src = st.gstart; bytes = sizeof(uint32_t) * st.P * (st.NG + 1); break;
            default: src = st.gend; bytes = sizeof(uint16_t) * st.P * st.NG * ara::kStreamGroupSlots; break;
        }
    } else {
        if (!layer) return fail(ARA_ERR_INVALID_ARG, "the fold's outputs need a layer");
        if (t->parts.P == 0) return fail(ARA_ERR_UNSUPPORTED, "the tables hold no partitioned copy (plain layout)");
        ara_layer probe = *layer;
        probe.trial_begin = 0;
        probe.trial_count = 0;
        ara::LayerArgs L;
        ara_status st = build_layer_args(t, probe, L);
        if (st != ARA_OK) return st;
        const size_t o_bytes = (sizeof(double) * t->C + 255) & ~size_t(255);
        const size_t p_bytes = static_cast<size_t>(ara::part_scratch_bytes(t->C, t->parts.P));
        HIP_TRY(buf.alloc(o_bytes + p_bytes, s), "scratch for the fold");
        double* o = static_cast<double*>(buf.p);
        void* pbuf = static_cast<char*>(buf.p) + o_bytes;
        HIP_TRY(ara::launch_fold_parts(t->sparse, t->C, L, nullptr, o, t->parts.P, pbuf, s), "fold and part images");
        if (what == ARA_DEBUG_OCCURRENCE) {
            src = o;
            bytes = sizeof(double) * t->C;
        } else if (what == ARA_DEBUG_IMAGES) {
            src = pbuf;
            bytes = ara::kImgPartBytes * t->parts.P;
        } else {
            const int64_t n_sb = static_cast<int64_t>(t->parts.P) * ara::kImgBase32;
            std::vector<uint32_t> cnt(n_sb);
            HIP_TRY(hipMemcpyAsync(cnt.data(), ara::part_superblock_counts(pbuf, t->parts.P), sizeof(uint32_t) * n_sb,
                                   hipMemcpyDeviceToHost, s),
                    "copy superblock counts");
            HIP_TRY(hipStreamSynchronize(s), "synchronize");
            int64_t nnz = 0;
            for (uint32_t c : cnt) nnz += c;
            src = ara::part_compact_values(pbuf, t->parts.P);
            bytes = sizeof(double) * nnz;
        }
    }
    *n_out = bytes;
    if (bytes > capacity) {
        HIP_TRY(hipStreamSynchronize(s), "synchronize");
        return fail(ARA_ERR_BUFFER_TOO_SMALL, "%lld bytes, capacity %lld", (long long)bytes, (long long)capacity);
    }
    if (bytes > 0) {
        if (!out) return fail(ARA_ERR_INVALID_ARG, "out is NULL");
        HIP_TRY(hipMemcpyAsync(out, src, bytes, hipMemcpyDeviceToHost, s), "copy");
    }
    HIP_TRY(hipStreamSynchronize(s), "synchronize");
    return ARA_OK;
}

ara_status ara_event_nets(ara_tables* t, const ara_layer* layer, double* nets, int64_t capacity, int64_t* n_out,
                          uint32_t flags, void* stream) {
    if (!t || !layer || !n_out || capacity < 0) return fail(ARA_ERR_INVALID_ARG, "NULL argument");
    ara::LayerArgs L;
    ara_status st = build_layer_args(t, *layer, L);
    if (st != ARA_OK) return st;
    DeviceScope ds(t->device);
    if (!ds.ok) return fail(ARA_ERR_DEVICE, "cannot select the tables' device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    UseFence use_fence(t, s);           // the tables' memory outlives this call's work
    int64_t be[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(&be[0], t->offsets + L.trial_begin, sizeof(int64_t), hipMemcpyDeviceToHost, s), "offsets");
    HIP_TRY(hipMemcpyAsync(&be[1], t->offsets + L.trial_begin + L.trial_count, sizeof(int64_t), hipMemcpyDeviceToHost,
                           s),
            "offsets");
    HIP_TRY(hipStreamSynchronize(s), "synchronize");
    const int64_t n = be[1] - be[0];
    *n_out = n;
    if (n > capacity) return fail(ARA_ERR_BUFFER_TOO_SMALL, "the layer's trials hold %lld events, capacity %lld",
                                  (long long)n, (long long)capacity);
    if (n == 0) return ARA_OK;
    if (!nets) return fail(ARA_ERR_INVALID_ARG, "NULL output");
    const bool dev = (flags & ARA_DEVICE_PTR) != 0;
    // kept scratch: o, the part images with the compact values, the probe
    // words, staged output
    auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
    const int P = ara::part_count(t->C);
    const size_t o_bytes = up(sizeof(double) * t->C);
    const size_t p_bytes = up(static_cast<size_t>(ara::part_scratch_bytes(t->C, P)));
    const size_t w_bytes = up(static_cast<size_t>(ara::probe_table_bytes(t->C)));
    const size_t n_bytes = dev ? 0 : up(sizeof(double) * n);
    ScratchLease lease(t->scratch_mu);
    lease.s = s;
    HIP_TRY(scratch_acquire(t->scratch_mu, t->scratch, o_bytes + p_bytes + w_bytes + n_bytes + 256, s, &lease.b),
            "scratch for occurrence losses, part images, probe words and net losses");
    char* base = static_cast<char*>(lease.b->p);
    uint64_t* probe = reinterpret_cast<uint64_t*>(base + o_bytes + p_bytes);
    double* out = dev ? nets : reinterpret_cast<double*>(base + o_bytes + p_bytes + w_bytes);
    HIP_TRY(ara::launch_fold_parts(t->sparse, t->C, L, nullptr, reinterpret_cast<double*>(base), P, base + o_bytes, s),
            "fold and part images");
    HIP_TRY(ara::launch_event_nets(t->offsets, t->ids, base + o_bytes, P, t->C, probe, L, out, t->n_cu, s),
            "net-loss kernel");
    if (!dev) {
        HIP_TRY(hipMemcpyAsync(nets, out, sizeof(double) * n, hipMemcpyDeviceToHost, s), "copy nets");
        HIP_TRY(hipStreamSynchronize(s), "synchronize");
    }
    return ARA_OK;
}

ara_status ara_read_checkpoints(ara_tables* t, int32_t what, double* out, int64_t capacity, int64_t* n_out) {
    if (!t || !n_out || (what != 0 && what != 1)) return fail(ARA_ERR_INVALID_ARG, "bad argument");
    std::lock_guard<std::mutex> g(t->mu);
    if (!t->ck.valid) return fail(ARA_ERR_NOT_READY, "no checkpointed forward");
    if (what == 1 && !t->ck.has_stride)
        return fail(ARA_ERR_NOT_READY, "no stride checkpoints (run with ARA_CHECKPOINT_STRIDE)");
    DeviceScope ds(t->device);
    const int64_t n = what == 0 ? t->ck.key.trial_count : t->n_events / ara::kStride;
    *n_out = n;
    if (capacity < n) return fail(ARA_ERR_BUFFER_TOO_SMALL, "need %lld values", (long long)n);
    if (n == 0) return ARA_OK;
    if (!out) return fail(ARA_ERR_INVALID_ARG, "NULL output");
    HIP_TRY(hipDeviceSynchronize(), "synchronize");
    HIP_TRY(hipMemcpy(out, what == 0 ? t->ck.S : t->ck.stride, sizeof(double) * n, hipMemcpyDeviceToHost), "copy");
    return ARA_OK;
}

}  // extern "C"
