/*
 * ara.h -- C ABI of the MI355X (gfx950) Aggregate Risk Analysis library.
 *
 * The analysis (Prades, Varghese, Reano, Silla, "Multi-Tenant Virtual GPUs
 * for Optimising Performance of a Financial Risk Application", Section IV)
 * maps a Year Event Table (YET, Eq. 1) and a set of Event Loss Tables (ELT,
 * Eq. 2) grouped into layers (Eq. 3) to a Year Loss Table (YLT): one loss per
 * trial, from which PML and TVaR are derived (Section IV-A, end).
 *
 * Per trial t, event occurrence d and layer ELT j (Algorithm 3):
 *     x_j  = clamp(ELT_j[E_{t,d}]; R_j, Lim_j)          per-ELT terms
 *     y_d  = sum_j x_j          (layer ELT order)        combine over ELTs
 *     o_d  = clamp(y_d; OccR, OccL)                       occurrence terms
 *     S_t  = sum_d o_d                                    annual total
 *     YLT_t= clamp(S_t; AggR, AggL)                       aggregate terms
 * with clamp(v; R, L) = min(max(v - R, 0), L).
 *
 * Conventions for every call:
 *   - Return value: ara_status, ARA_OK (0) on success.  On failure nothing
 *     observable has been written to outputs, and ara_last_error() returns a
 *     thread-local message.  No exception or abort crosses this ABI.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Pointers are host memory unless ARA_DEVICE_PTR is set in `flags`, in
 *     which case the pointers named by that call's comment are device memory
 *     on the device the tables live on.  ara_layer arrays are always host.
 *   - Calls with host outputs return after the results are in host memory.
 *     Calls with device outputs are asynchronous on `stream`.
 *   - Tables are read-only after creation: several threads may run layers on
 *     the same tables concurrently, on different streams.  The scratch of
 *     ara_run_layers (per-layer sequences), ara_run_portfolio, ara_event_nets
 *     and ara_risk_metrics is device memory kept between calls (by the
 *     tables, or by the library per device for the metrics): a call reuses a
 *     buffer last used on its own stream at once, one last used on another
 *     stream once that stream has passed its last use, and otherwise
 *     allocates a new one.  Other scratch, staging for host arguments and
 *     the tables' own copies come from the library's device memory cache
 *     (memory from hipMalloc, kept when freed and handed out again under the
 *     same stream rule), so steady-state calls neither allocate from nor
 *     return memory to the runtime.  Destroying tables returns their memory to
 *     the cache after the last work enqueued on them, without waiting.
 */
#ifndef ARA_H
#define ARA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ara_status;

#define ARA_OK                   0
#define ARA_ERR_INVALID_ARG      1  /* malformed argument: NULL, negative size, NaN term, p outside (0,1), bad CSR */
#define ARA_ERR_OUT_OF_RANGE     2  /* an event ID >= catalogue size, or an ELT index outside the pool */
#define ARA_ERR_BUFFER_TOO_SMALL 3  /* an output capacity is below what the call writes */
#define ARA_ERR_NO_MEMORY        4  /* a device or pinned-host allocation failed */
#define ARA_ERR_DEVICE           5  /* a HIP runtime error; the HIP message is in ara_last_error() */
#define ARA_ERR_NOT_READY        6  /* ara_backward without a matching checkpointed forward */
#define ARA_ERR_UNSUPPORTED      7  /* a valid request the library does not handle (e.g. J > ARA_MAX_LAYER_ELTS) */

/* flags */
#define ARA_DEVICE_PTR   (1u << 0)  /* pointer arguments of the call are device memory */
#define ARA_LITERAL      (1u << 1)  /* ara_run_layers: per-occurrence, per-ELT lookups exactly as
                                       Algorithm 3 is written, instead of one lookup of the
                                       per-event occurrence loss computed for the whole catalogue */
#define ARA_CHECKPOINT_S (1u << 2)  /* ara_run_layers: keep each trial's annual total S_t and
                                       YLT_t inside the tables for ara_backward */
#define ARA_PER_LAYER    (1u << 3)  /* ara_run_layers with several layers and pass_variant 1: one
                                       launch sequence per layer instead of the batched launch (a
                                       fold per layer, then one persistent pass over a (layer, tile)
                                       work list sorted by decreasing cost).  With pass_variant 0
                                       (the default) or 2 layers always run one sequence each. */
#define ARA_GRAPH        (1u << 4)  /* ara_run_layers: replay a HIP graph of the whole call, captured
                                       on first use for this shape (layer count, trial ranges,
                                       output pointer; with pass_variant 1 also the ELT counts) --
                                       the per-layer sequences, or with pass_variant 1 and several
                                       layers the batched launch.  Terms and ELT choices may change
                                       between replays (they are copied to the device only when
                                       they differ from the last replay's, so repeated replays
                                       queue without host waits).  Requires a
                                       device output and a non-null stream (ARA_ERR_INVALID_ARG
                                       otherwise). */
#define ARA_PROFILE      (1u << 5)  /* ara_run_layers: bracket each kernel with HIP events on the
                                       call's stream; read the totals with ara_kernel_stats */

#define ARA_CHECKPOINT_STRIDE (1u << 7) /* ara_run_layers: ARA_CHECKPOINT_S plus the prefix sums
                                       of S every 64 events in time order (read them with
                                       ara_read_checkpoints); the default pass and pass_variant
                                       2 add one time-ordered pass over the 32-bit YET for them,
                                       pass_variant 1 runs the time-ordered trial pass instead */
#define ARA_PLAIN_LAYOUT (1u << 6)  /* ara_create_tables: keep only the time-ordered YET (no
                                       catalogue-partitioned copy; saves ~4 B per event of device
                                       memory, slower ara_run_layers) */

/* kernel classes reported by ara_kernel_stats */
#define ARA_KERNEL_FOLD       0     /* per-catalogue occurrence losses */
#define ARA_KERNEL_TRIAL_PASS 1     /* YET stream, lookups, annual totals, aggregate terms */
#define ARA_KERNEL_BATCHED    2     /* persistent multi-layer trial pass */
#define ARA_KERNEL_COMBINE    3     /* merge of the per-part partial sums into annual totals and
                                       aggregate terms (after the catalogue-partitioned pass) */
#define ARA_KERNEL_AGGREGATE  4     /* per-trial program and portfolio sums of layer year losses */

#define ARA_MAX_LAYER_ELTS 64       /* most ELTs one layer may cover (the paper's layers cover 3-30) */
#define ARA_CHECKPOINT_EVERY 64     /* events between stored prefix sums of S */
#define ARA_MAX_PROGRAMS 64         /* most programs one ara_run_portfolio call takes (the
                                       paper's portfolios hold 1-10) */

typedef struct ara_tables ara_tables;

/*
 * A layer (Eq. 3): the ELTs it covers and its terms.  The per-ELT terms
 * (the tuple attached to each ELT in Eq. 2) are read as a retention and a
 * limit.  The layer terms are (OccR, OccL, AggR, AggL).  All arrays are host
 * memory, n_elts entries, in the layer's ELT order (the order in which x_j
 * are summed).  Retentions >= 0, limits >= 0 (+inf allowed), no NaN.
 * The layer covers trials [trial_begin, trial_begin + trial_count).
 */
typedef struct ara_layer {
    int32_t n_elts;
    const int32_t* elt_index;       /* rows of the ELT pool */
    const double* elt_retention;
    const double* elt_limit;
    double occ_retention, occ_limit;
    double agg_retention, agg_limit;
    int64_t trial_begin, trial_count;
} ara_layer;

/*
 * A program (Section IV-A): the layers it covers, in order.  `layers` is
 * host memory holding n_layers entries.
 */
typedef struct ara_program {
    int32_t n_layers;
    const ara_layer* layers;
} ara_program;

/*
 * Outputs of ara_run_portfolio.  Each pointer may be NULL to skip that
 * output; the capacities count doubles.  With n = the portfolio's trial
 * count and the layers numbered across programs in order:
 *   layer_ylt      [n_layers_total][n]: the layers' year losses;
 *   program_ylt    [n_programs][n]: per trial, the sum of the program's layers;
 *   portfolio_ylt  [n]: per trial, the sum of every layer of the portfolio.
 */
typedef struct ara_portfolio_out {
    double* layer_ylt;
    int64_t layer_capacity;
    double* program_ylt;
    int64_t program_capacity;
    double* portfolio_ylt;
    int64_t portfolio_capacity;
} ara_portfolio_out;

/*
 * Launch-shape knobs picked by the autotuner; zero fields mean "default".
 */
typedef struct ara_tuning {
    int32_t block_threads;          /* reserved (0); workgroup sizes are fixed per kernel */
    int32_t part_lanes_per_trial;   /* partitioned passes: lanes per trial group, 8/16/32/64
                                       (0 = 16; the XCD-affine pass takes 8/16/32, 0 or 64 = 8) */
    int32_t lanes_per_trial;        /* time-ordered pass: 64 (one wave per trial), 32, 16 or 8 */
    int32_t blocks_per_cu;          /* time-ordered pass: resident workgroups per CU (0 = 8) */
    int32_t fold_events_per_thread; /* reserved (0) */
    int32_t schedule;               /* batched pass work order: 0 = decreasing cost, 1 = layer-major */
    int32_t pass_variant;           /* pass over the YET: 0 = the 16-bit part-major copy streamed
                                       against per-part LDS byte maps and loss copies (falls back
                                       to 2 when the tables hold no such copy), 1 = the 32-bit
                                       partitioned copy with LDS ranks + compact values, one
                                       persistent launch for several layers, 2 = the 32-bit
                                       partitioned copy, each XCD serving its own catalogue parts.
                                       ara_backward's histogram follows it: 0 over the 16-bit copy,
                                       1 and 2 over the 32-bit copy */
    int32_t reserved;
} ara_tuning;

/*
 * ara_create_tables -- Algorithm 2 (TransferDataToDevice): make the YET and
 * the ELT pool resident on the current device.
 *
 *   trial_offsets  int64[n_trials + 1], CSR offsets: trial t's events are
 *                  event_ids[trial_offsets[t] .. trial_offsets[t+1]), in
 *                  ascending time-stamp order (Eq. 1).  offsets[0] == 0,
 *                  non-decreasing, offsets[n_trials] == n_events.
 *   event_ids      uint32[n_events], catalogue indices < catalogue_size.
 *   elt_losses     float64[n_elts][catalogue_size], row-major dense
 *                  direct-access tables (Section IV-B); 0.0 = no loss.
 *                  Finite and >= 0.
 *   flags          ARA_DEVICE_PTR: the three arrays are device memory.
 *                  ARA_PLAIN_LAYOUT: skip the catalogue-partitioned copies.
 *
 * Besides the time-ordered CSR the library keeps, by default, two more
 * copies of the event IDs laid out for its trial passes.  The 32-bit
 * partitioned copy: tiles of 256 consecutive trials, inside a tile the
 * catalogue's parts of 2^18 events one after the other, inside a part each
 * trial's events of that part in time order.  The 16-bit copy, which the
 * default pass streams: the catalogue cut into parts of 2^16 events, and per
 * part one stream of part-relative IDs holding, group of consecutive trials
 * after group, each trial's events of that part in time order (about 2 bytes
 * per event).  Both depend on the YET alone, so every layer run on the
 * tables uses them (ara_layout_info_get reports their sizes).
 *   out            receives the handle; freed by ara_destroy_tables.
 *
 * The arrays are caller-owned and only read during the call: the library
 * copies them into device memory it owns.  Validation runs on the device
 * after the copy: ARA_ERR_OUT_OF_RANGE for an ID >= catalogue_size,
 * ARA_ERR_INVALID_ARG for bad offsets or a negative/NaN/inf loss,
 * ARA_ERR_NO_MEMORY if the device cannot hold the tables.  Synchronous.
 */
ara_status ara_create_tables(const int64_t* trial_offsets, int64_t n_trials,
                             const uint32_t* event_ids, int64_t n_events,
                             const double* elt_losses, int32_t n_elts,
                             int64_t catalogue_size, uint32_t flags, void* stream,
                             ara_tables** out);

/*
 * ara_create_yet -- Algorithm 2 for one YET slice when the ELTs are already
 * resident: new tables that own the given YET (copied like ara_create_tables
 * does, validated against base's catalogue, with the partitioned copy unless
 * ARA_PLAIN_LAYOUT) and share base's ELT pool without copying it.  `base`
 * must outlive the new tables.  Errors as ara_create_tables.
 */
ara_status ara_create_yet(const ara_tables* base, const int64_t* trial_offsets, int64_t n_trials,
                          const uint32_t* event_ids, int64_t n_events, uint32_t flags, void* stream,
                          ara_tables** out);

/* Release the device memory of the tables.  NULL is accepted. */
void ara_destroy_tables(ara_tables* tables);

/*
 * ara_run_layers -- Algorithm 1's layer loop around Algorithm 3: the year
 * loss of every trial of every layer.
 *
 *   layers/n_layers  host array of layer descriptions (see ara_layer).
 *   ylt              float64 output, the layers' year losses back to back
 *                    (layer 0's trial_count values first); host memory, or
 *                    device memory with ARA_DEVICE_PTR.
 *   ylt_capacity     number of doubles `ylt` can hold; ARA_ERR_BUFFER_TOO_SMALL
 *                    if below the sum of trial_count.
 *   flags            ARA_DEVICE_PTR, ARA_LITERAL, ARA_CHECKPOINT_S or
 *                    ARA_CHECKPOINT_STRIDE (one layer only), ARA_PER_LAYER,
 *                    ARA_GRAPH, ARA_PROFILE.
 *
 * Year losses do not depend on the flags beyond floating-point rounding of
 * S (the sum over occurrences is accumulated in double-double and rounded
 * once, so it equals the correctly rounded sum except within ~1e-29 relative
 * of a rounding tie).  Errors: ARA_ERR_INVALID_ARG (negative/NaN term, bad
 * trial range), ARA_ERR_OUT_OF_RANGE (ELT index outside the pool),
 * ARA_ERR_UNSUPPORTED (n_elts > ARA_MAX_LAYER_ELTS).
 */
ara_status ara_run_layers(ara_tables* tables, const ara_layer* layers, int32_t n_layers,
                          double* ylt, int64_t ylt_capacity, uint32_t flags, void* stream);

/*
 * ara_risk_metrics -- the portfolio risk metrics named in Section IV-A
 * (PML, TVaR), plus the mean annual loss, from one layer's YLT.
 *
 *   ylt        float64[n_trials], values >= 0 (as produced by ara_run_layers);
 *              host memory or device memory with ARA_DEVICE_PTR.
 *   probs      host float64[n_probs], each in (0, 1); n_probs <= 4
 *              (ARA_ERR_UNSUPPORTED above).
 *   mean_out   1 double; pml_out, tvar_out n_probs doubles each; host
 *              memory, or device memory with ARA_DEVICE_PTR.
 *
 * With m = ara_tail_count(n_trials, p) (below): PML_p is the m-th largest
 * year loss and TVaR_p the mean of the m largest.  Sums are accumulated in
 * double-double and rounded once.  Errors: ARA_ERR_INVALID_ARG for
 * n_trials < 1 or p outside (0, 1).
 */
ara_status ara_risk_metrics(const double* ylt, int64_t n_trials, const double* probs,
                            int32_t n_probs, double* mean_out, double* pml_out,
                            double* tvar_out, uint32_t flags, void* stream);

/*
 * ara_analyze -- one layer's year losses and its risk metrics in one call:
 * the results of ara_run_layers(tables, layer, 1, ylt, ...) followed by
 * ara_risk_metrics over those year losses, bit for bit (the same kernels).
 *
 *   layer       as ara_run_layers (one layer, trial_count >= 1).
 *   probs       host float64[n_probs], each in (0, 1); n_probs <= 4.
 *   ylt         float64[trial_count] (ylt_capacity values at least).
 *   metrics     float64[1 + 2 * n_probs]: the mean, then PML_p for each p,
 *               then TVaR_p for each p.
 *   flags       ARA_DEVICE_PTR (ylt and metrics are device memory),
 *               ARA_GRAPH (with ARA_DEVICE_PTR and a non-null stream: the
 *               fold, the pass, the combine and the metrics kernels are
 *               captured as one HIP graph per output addresses, trial range
 *               and tail counts, with scratch of its own, and replayed; new
 *               terms and ELT choices reuse it), ARA_PROFILE.
 *
 * Errors as ara_run_layers and ara_risk_metrics; ARA_ERR_INVALID_ARG for
 * other flags.  Asynchronous on `stream` with device outputs.
 */
ara_status ara_analyze(ara_tables* tables, const ara_layer* layer, const double* probs, int32_t n_probs,
                       double* ylt, int64_t ylt_capacity, double* metrics, uint32_t flags, void* stream);

/*
 * ara_risk_metrics_noalloc -- for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same results as ara_risk_metrics with ARA_DEVICE_PTR, from
 * the same kernels, but the scratch they need lives in a static device array
 * of the library (one per device, held until the process ends) instead of
 * memory the call allocates.  The call allocates nothing, host or device.
 *
 *   ylt        device float64[n_trials], values >= 0.
 *   probs      host float64[n_probs], each in (0, 1); n_probs <= 4.
 *   mean_out, pml_out, tvar_out   device memory (1, n_probs and n_probs
 *              doubles), written on `stream` without waiting.
 *
 * Limit: n_probs * n_trials <= ARA_METRICS_NOALLOC_KEYS (any n_trials for
 * n_probs = 0), else ARA_ERR_UNSUPPORTED before any device work.  Every call
 * on one device uses that device's one array, so calls that overlap in time
 * on one device race and give wrong results: order them (one stream, or
 * events).  Other errors as ara_risk_metrics.
 */
#define ARA_METRICS_NOALLOC_KEYS (4ll << 20)
ara_status ara_risk_metrics_noalloc(const double* ylt, int64_t n_trials, const double* probs,
                                    int32_t n_probs, double* mean_out, double* pml_out,
                                    double* tvar_out, void* stream);

/*
 * ara_backward -- gradients of the mean annual loss and of TVaR_p with
 * respect to theta = [R_1..R_J, Lim_1..Lim_J, OccR, OccL, AggR, AggL] of one
 * layer (2J + 4 values each, in that order).  The paper defines no
 * gradient; the year loss is piecewise linear in theta and the convention at
 * a kink is the strict one: a clamp with reduced value t = v - R passes the
 * slope only for 0 < t < L, d/dR = -1 there, d/dL = 1 for t > L, 0 at equality.
 * Every partial is then an integer count; the mean divides by n, TVaR by m
 * (trials tied at the m-th largest value share the remaining slots equally).
 *
 * Requires a preceding ara_run_layers(tables, layer, 1, ..., ARA_CHECKPOINT_S)
 * with identical layer terms, else ARA_ERR_NOT_READY.  grad_mean/grad_tvar
 * are host memory (2J + 4 doubles each), or device memory with
 * ARA_DEVICE_PTR.  Either may be NULL to skip it.  The per-event occurrence
 * counts come from one pass over the YET: with pass_variant 0 (the default)
 * over the 16-bit part-major copy, else over the 32-bit partitioned copy
 * (the plain layout's own pass without either); all give the same integers.
 */
ara_status ara_backward(ara_tables* tables, const ara_layer* layer, double tvar_p,
                        double* grad_mean, double* grad_tvar, uint32_t flags, void* stream);

/* ------------------------------------------------------------------------ */
/* auxiliary calls                                                          */
/* ------------------------------------------------------------------------ */

/* Thread-local message describing the last failure on this thread. */
const char* ara_last_error(void);

/* Static name of a status code. */
const char* ara_status_string(ara_status status);

/* Device bytes held by the tables (YET, offsets, ELT pool). */
ara_status ara_table_bytes(const ara_tables* tables, int64_t* bytes);

/*
 * The library's device memory cache on the current device (see the
 * threading notes at the top): memory freed by tables and calls stays cached
 * for reuse instead of going back to the runtime.
 *
 * ara_cached_memory -- bytes the cache holds in total, and of those the
 *   bytes no tables or call is using (idle).  Either pointer may be NULL.
 * ara_release_cached_memory -- returns to the runtime (hipFree, which waits
 *   for the device) every idle block whose last use has completed, for
 *   callers that need the memory elsewhere; reports the bytes released
 *   (NULL: not reported).  Blocks in use, or whose last use is still running,
 *   stay cached.  Later calls allocate again as needed.
 */
ara_status ara_cached_memory(int64_t* held_bytes, int64_t* idle_bytes);
ara_status ara_release_cached_memory(int64_t* bytes_released);

/* Peak device scratch bytes ara_run_layers(tables, layers, n_layers, ..,
   flags) allocates beyond the tables and the output; for admission control. */
ara_status ara_footprint(const ara_tables* tables, const ara_layer* layers, int32_t n_layers,
                         uint32_t flags, int64_t* bytes);

/*
 * Device bytes, for admission control (upper bounds, computed on the host):
 * ara_yet_footprint     -- the peak that ara_create_tables (without its ELT
 *                          pool) or ara_create_yet holds for a YET of these
 *                          sizes with `flags` (ARA_PLAIN_LAYOUT: no
 *                          partitioned copies), its build temporaries included;
 * ara_metrics_footprint -- the scratch of one ara_risk_metrics call over
 *                          n_trials year losses and n_probs probabilities
 *                          (with ARA_DEVICE_PTR: device inputs and outputs).
 * Together with ara_footprint (an ara_run_layers call's scratch) they give
 * what one analysis adds to the device on top of the resident tables.
 */
ara_status ara_yet_footprint(int64_t n_trials, int64_t n_events, int64_t catalogue_size, uint32_t flags,
                             int64_t* bytes);
ara_status ara_metrics_footprint(int64_t n_trials, int32_t n_probs, uint32_t flags, int64_t* bytes);

/*
 * ara_debug_lookups -- the raw lookups of Algorithm 3 for one trial, as the
 * device performs them: ids_out[k] = k-th event ID of the trial and
 * losses_out[k * n_elts + j] = ELT_{elt_index[j]}[ids_out[k]].  Host outputs;
 * `capacity` is the number of events the buffers hold (losses_out holds
 * capacity * n_elts doubles); *n_out receives the trial's event count.
 * ARA_ERR_BUFFER_TOO_SMALL if the trial has more events than `capacity`.
 */
ara_status ara_debug_lookups(ara_tables* tables, const ara_layer* layer, int64_t trial,
                             uint32_t* ids_out, double* losses_out, int64_t capacity,
                             int64_t* n_out, void* stream);

/*
 * ara_debug_read -- the data the default pass works from, copied to host for
 * bit-exact checks of its lookups and indexing (Algorithm 3's lookup step;
 * Section IV-B: direct-access tables).  `what`:
 *   ARA_DEBUG_OCCURRENCE     float64[C]: o(E) for every catalogue event E (the
 *                            per-ELT terms, the sum over the layer's ELTs in
 *                            layer order, the occurrence terms), as the fold
 *                            of `layer` writes it for the pass
 *   ARA_DEBUG_COMPACT        float64[nnz]: the nonzero o(E) in catalogue order,
 *                            the array the pass reads them from by rank
 *   ARA_DEBUG_IMAGES         uint8[image_parts * 37120]: per 2^18-event part,
 *                            4096 u64 bitmap words of o(E) != 0 (bit E % 64
 *                            of word E / 64), 2048 u16 counts of nonzero events
 *                            before each 128-event block inside its
 *                            4096-event superblock, 64 u32 global ranks of
 *                            each superblock's first nonzero event
 *   ARA_DEBUG_STREAM_IDS     uint16[stream_ids]: the 16-bit copy of the YET
 *                            (see ara_create_tables and ara_layout_info_get)
 *   ARA_DEBUG_STREAM_BASE    int64[stream_parts + 1]: where each part's stream starts
 *   ARA_DEBUG_STREAM_GSTART  uint32[stream_parts][stream_groups + 1]: group
 *                            starts relative to the part's stream
 *   ARA_DEBUG_STREAM_GEND    uint16[stream_parts][stream_groups][64]: end of
 *                            each trial of the group relative to the group's
 *                            start (slots past the group's trials repeat its end)
 * `layer` (its trial range is ignored) is needed for the first three only.
 * `out` is host memory of `capacity` bytes; *n_out receives the bytes of the
 * result (ARA_ERR_BUFFER_TOO_SMALL, nothing copied, if above capacity).
 * ARA_ERR_UNSUPPORTED when the tables hold no such copy.  Synchronous.
 */
#define ARA_DEBUG_OCCURRENCE    0
#define ARA_DEBUG_COMPACT       1
#define ARA_DEBUG_IMAGES        2
#define ARA_DEBUG_STREAM_IDS    3
#define ARA_DEBUG_STREAM_BASE   4
#define ARA_DEBUG_STREAM_GSTART 5
#define ARA_DEBUG_STREAM_GEND   6
ara_status ara_debug_read(ara_tables* tables, const ara_layer* layer, int32_t what, void* out,
                          int64_t capacity, int64_t* n_out, void* stream);

/*
 * ara_run_portfolio -- Algorithm 1: for each program of the portfolio PF
 * (Section IV-A), for each of its layers, the YET split into n_splits
 * contiguous trial ranges YET_i, each analysed as its own launch sequence,
 * and the layer's YLT populated from the parts.  The paper gives no rule for
 * combining layers; a program's year loss is read as the per-trial sum of
 * its layers' year losses, the portfolio's as the sum over all its layers
 * (no terms above the layer).  Both sums are accumulated in double-double
 * in layer order and rounded once.
 *
 *   programs   n_programs entries (1..ARA_MAX_PROGRAMS), each with >= 1 layer.
 *              Every layer must cover the same trials (same trial_begin and,
 *              after resolving -1, the same count): the portfolio's range.
 *   n_splits   >= 1.  Split i covers trials [b_i, b_{i+1}) with
 *              b_i = begin + floor(i * n / n_splits); empty splits are skipped.
 *              Results do not depend on n_splits (trials are independent).
 *   out        see ara_portfolio_out; capacities too small give
 *              ARA_ERR_BUFFER_TOO_SMALL (nothing written).
 *   flags      ARA_DEVICE_PTR (all output pointers are device memory; the
 *              call returns without waiting), ARA_LITERAL, ARA_PROFILE
 *              (ARA_KERNEL_AGGREGATE times the sums).
 * ARA_ERR_INVALID_ARG for layers over different trials, n_splits < 1 or no
 * output; ARA_ERR_UNSUPPORTED beyond ARA_MAX_PROGRAMS.
 */
ara_status ara_run_portfolio(ara_tables* tables, const ara_program* programs, int32_t n_programs,
                             int32_t n_splits, const ara_portfolio_out* out, uint32_t flags, void* stream);

/*
 * ara_event_nets -- per-event net losses of one layer, the cumulative form of
 * the aggregate terms (Section IV-B: the aggregate terms act on the
 * cumulative loss of the trial).  For each trial t of the layer and its
 * events d = 1..K_t in storage (time) order, with S_d the running total of
 * the occurrence losses o and A_d = clamp(S_d; AggR, AggL), A_0 =
 * clamp(0; AggR, AggL):  nets[i] = A_d - A_{d-1}, where i is the event's
 * position counted from the first event of the layer's first trial.  Each
 * S_d is rounded once from an extended-precision running sum.  The nets of a
 * trial add up to its year loss minus A_0.
 *
 *   nets      float64[capacity]; host memory, or device memory with
 *             ARA_DEVICE_PTR (then written on `stream` without waiting).
 *   *n_out    receives the number of events in the layer's trials.
 * ARA_ERR_BUFFER_TOO_SMALL if capacity < *n_out (nothing written).
 */
ara_status ara_event_nets(ara_tables* tables, const ara_layer* layer, double* nets, int64_t capacity,
                          int64_t* n_out, uint32_t flags, void* stream);

/*
 * ara_read_checkpoints -- copy the state kept by ARA_CHECKPOINT_S (what = 0)
 * or ARA_CHECKPOINT_STRIDE (what = 1) to host.
 * what = 0: S_t for the layer's trials (trial_count doubles);
 * what = 1: stride-64 prefix checkpoints: slot b holds, for the trial that
 *           owns global event 64b+63, the sum of o over that trial's events
 *           up to and including event 64b+63 (n_events/64 doubles; slots
 *           whose event lies outside the layer's trials hold NaN).
 * *n_out receives the number of values.
 */
ara_status ara_read_checkpoints(ara_tables* tables, int32_t what, double* out,
                                int64_t capacity, int64_t* n_out);

/*
 * ara_kernel_stats -- launches and summed device time (ms, from HIP events)
 * of one kernel class (ARA_KERNEL_*, 0..4; ARA_ERR_INVALID_ARG otherwise)
 * over the ara_run_layers and ara_run_portfolio calls made with ARA_PROFILE
 * since the last reset.
 * With the catalogue-partitioned pass, ARA_KERNEL_TRIAL_PASS times the pass
 * kernel alone and ARA_KERNEL_COMBINE the merge after it.  Waits for the
 * recorded events.  reset != 0 clears the totals after reading them.
 */
ara_status ara_kernel_stats(ara_tables* tables, int32_t kernel, int64_t* launches, double* total_ms,
                            int32_t reset);

/* Launch-shape knobs used by later calls on these tables (NULL resets). */
ara_status ara_set_tuning(ara_tables* tables, const ara_tuning* tuning);
ara_status ara_get_tuning(const ara_tables* tables, ara_tuning* tuning);

/*
 * ara_tail_count -- the number m of largest year losses that PML_p and
 * TVaR_p are taken over (Section IV-A names both metrics without defining
 * them).  m = ceil(n_trials * (1 - p)) with p read as the decimal it was
 * written as: the shortest decimal string that converts back to the same
 * double, taken exactly (so p = 0.99 gives m = 10000 for 10^6 trials, and
 * p = 0.989999999999 gives 10001), then clamped to [1, n_trials].  Host
 * only; needs no device.  ARA_ERR_INVALID_ARG for n_trials < 1, p outside
 * (0, 1) or m NULL.  ara_risk_metrics and ara_backward use this m.
 */
ara_status ara_tail_count(int64_t n_trials, double p, int64_t* m);

/*
 * The device copies of the YET the tables keep for their passes, for
 * measurement (the bytes a pass streams) and admission control.
 *   image_parts          catalogue parts of 2^18 events (the per-request part
 *                        images and the 32-bit partitioned copy); 0 if the
 *                        partitioned copy is absent
 *   partitioned_ids      32-bit IDs in the partitioned copy, padding included
 *   stream_parts         catalogue parts of 2^16 events of the 16-bit copy
 *                        that the default pass streams; 0 if absent
 *   stream_group_trials  trials per group of that copy
 *   stream_groups        groups per part (ceil(n_trials / stream_group_trials))
 *   stream_ids           16-bit IDs in that copy, padding included
 *   *_bytes              device bytes of each copy with its offsets
 */
typedef struct ara_layout_info {
    int32_t image_parts;
    int32_t stream_parts;
    int32_t stream_group_trials;
    int32_t reserved;
    int64_t partitioned_ids;
    int64_t partitioned_bytes;
    int64_t stream_groups;
    int64_t stream_ids;
    int64_t stream_bytes;
} ara_layout_info;
ara_status ara_layout_info_get(const ara_tables* tables, ara_layout_info* info);

/* Number of compute units and the device index of the tables' device. */
ara_status ara_device_info(int32_t* n_cu, int32_t* device);

#ifdef __cplusplus
}
#endif

#endif /* ARA_H */
