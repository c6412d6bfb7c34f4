/*
 * ara_oracle.c -- CPU oracle for Aggregate Risk Analysis.  TEST
 * INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
 * baseline call it; the GPU library never does.
 *
 * Plain FP64 C, written from the paper's description of the analysis
 * (Section IV-B, Algorithm 3 and the term definitions that follow it):
 *
 *   for every trial T of the Year Event Table (Eq. 1), in storage order
 *     for every event E of T, in ascending time-stamp order
 *       for every ELT covered by the layer, in layer order
 *         look E up in the direct-access ELT (Eq. 2)     -> l
 *         apply the ELT's financial terms                -> x = clamp(l; R, Lim)
 *         add x to the event's layer loss                -> y += x
 *       apply the occurrence terms to the occurrence     -> o = clamp(y; OccR, OccL)
 *       accumulate the occurrence into the year          -> S += o
 *     apply the aggregate terms to the year's total      -> YLT = clamp(S; AggR, AggL)
 *
 * with clamp(v; R, L) = min(max(v - R, 0), L).  The paper prints "max" with a
 * single argument; the reading max(v - R, 0) is the only one under which a
 * retention removes loss and the result stays in [0, L].
 *
 * Summation of S: Algorithm 3 accumulates in time order.  The year loss is
 * by definition the sum of the occurrence-net losses, so besides the
 * sequential FP64 sum (SUM_SEQUENTIAL, the order as written) the oracle
 * offers that sum rounded once to FP64 (SUM_EXACT), computed with
 * Shewchuk's exact non-overlapping partials (Shewchuk 1997, "Adaptive
 * Precision Floating-Point Arithmetic"), the method behind Python's
 * math.fsum.  SUM_EXACT is the parity reference.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 * Trials are independent, so OpenMP splits trials only; each trial is
 * evaluated sequentially.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_ERR_RANGE 1
#define ORACLE_ERR_ARG 2

#define SUM_SEQUENTIAL 0
#define SUM_EXACT 1

/* ---------------------------------------------------------------------- */
/* financial terms                                                         */
/* ---------------------------------------------------------------------- */

/* clamp(v; r, lim) = min(max(v - r, 0), lim): a retention r then a limit lim */
static double apply_terms(double v, double r, double lim)
{
    double t = v - r;
    if (!(t > 0.0)) t = 0.0;
    if (t > lim) t = lim;
    return t;
}

/* ---------------------------------------------------------------------- */
/* exact summation: non-overlapping partials, rounded once at the end      */
/* ---------------------------------------------------------------------- */

#define MAX_PARTIALS 80

typedef struct {
    double p[MAX_PARTIALS];
    int n;
} exact_sum;

static void exact_init(exact_sum* a) { a->n = 0; }

static void exact_add(exact_sum* a, double x)
{
    int i = 0;
    for (int k = 0; k < a->n; ++k) {
        double y = a->p[k];
        if (fabs(x) < fabs(y)) { double t = x; x = y; y = t; }
        double hi = x + y;
        double lo = y - (hi - x);
        if (lo != 0.0) a->p[i++] = lo;
        x = hi;
    }
    a->p[i] = x;
    a->n = i + 1;
}

static double exact_result(const exact_sum* a)
{
    int n = a->n;
    double hi = 0.0, lo = 0.0;
    if (n > 0) {
        hi = a->p[--n];
        while (n > 0) {
            double x = hi;
            double y = a->p[--n];
            hi = x + y;
            double yr = hi - x;
            lo = y - yr;
            if (lo != 0.0) break;
        }
        /* round-half-even correction when the rest of the partials push the
           discarded part past a half-way point */
        if (n > 0 && ((lo < 0.0 && a->p[n - 1] < 0.0) || (lo > 0.0 && a->p[n - 1] > 0.0))) {
            double y = lo * 2.0;
            double x = hi + y;
            double yr = x - hi;
            if (y == yr) hi = x;
        }
    }
    return hi;
}

/* exported so the tests can compare it with math.fsum */
double ara_oracle_exact_sum(const double* x, int64_t n)
{
    exact_sum a;
    exact_init(&a);
    for (int64_t i = 0; i < n; ++i) exact_add(&a, x[i]);
    return exact_result(&a);
}

/* ---------------------------------------------------------------------- */
/* one occurrence: lookups + ELT terms + ELT sum + occurrence terms        */
/* ---------------------------------------------------------------------- */

typedef struct {
    const double* elts;        /* pool, row-major [n_pool][C] */
    int64_t C;
    int32_t J;
    const int32_t* elt_index;  /* layer's pool rows, layer order */
    const double* R;
    const double* Lim;
    double occR, occL;
} layer_view;

static double occurrence_loss(const layer_view* L, uint32_t e, double* y_out)
{
    double y = 0.0;
    for (int32_t j = 0; j < L->J; ++j) {
        double l = L->elts[(int64_t)L->elt_index[j] * L->C + (int64_t)e];
        y = y + apply_terms(l, L->R[j], L->Lim[j]);
    }
    if (y_out) *y_out = y;
    return apply_terms(y, L->occR, L->occL);
}

static int check_layer(const layer_view* L, int32_t n_pool)
{
    if (L->J < 0) return ORACLE_ERR_ARG;
    for (int32_t j = 0; j < L->J; ++j)
        if (L->elt_index[j] < 0 || L->elt_index[j] >= n_pool) return ORACLE_ERR_RANGE;
    return ORACLE_OK;
}

/* ---------------------------------------------------------------------- */
/* Algorithm 3 for one layer over a range of trials                        */
/* ---------------------------------------------------------------------- */

int ara_oracle_run_layer(const int64_t* offsets, int64_t n_trials,
                         const uint32_t* ids, int64_t n_events,
                         const double* elts, int32_t n_pool, int64_t C,
                         int32_t J, const int32_t* elt_index,
                         const double* R, const double* Lim,
                         double occR, double occL, double aggR, double aggL,
                         int64_t trial_begin, int64_t trial_count,
                         int32_t sum_mode, double* ylt_out, double* s_out,
                         int32_t n_threads)
{
    layer_view L = {elts, C, J, elt_index, R, Lim, occR, occL};
    if (check_layer(&L, n_pool) != ORACLE_OK) return ORACLE_ERR_RANGE;
    if (trial_begin < 0 || trial_count < 0 || trial_begin + trial_count > n_trials)
        return ORACLE_ERR_ARG;
    if (offsets[n_trials] != n_events) return ORACLE_ERR_ARG;
    int bad = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t k = 0; k < trial_count; ++k) {
        int64_t t = trial_begin + k;
        double S = 0.0;
        exact_sum acc;
        exact_init(&acc);
        for (int64_t i = offsets[t]; i < offsets[t + 1]; ++i) {
            uint32_t e = ids[i];
            if ((int64_t)e >= C) { bad |= 1; continue; }
            double o = occurrence_loss(&L, e, NULL);
            if (sum_mode == SUM_EXACT) exact_add(&acc, o);
            else S = S + o;
        }
        if (sum_mode == SUM_EXACT) S = exact_result(&acc);
        if (s_out) s_out[k] = S;
        ylt_out[k] = apply_terms(S, aggR, aggL);
    }
    return bad ? ORACLE_ERR_RANGE : ORACLE_OK;
}

/*
 * Per-event net losses: the aggregate terms act on the trial's cumulative
 * loss (Section IV-B), so after the d-th event of a trial (time order) the
 * recovered amount is A_d = clamp(S_d; AggR, AggL) with S_d the sum of the
 * first d occurrence losses, and the d-th event adds A_d - A_{d-1}, with
 * A_0 = clamp(0; AggR, AggL).  Each S_d is the exact running sum rounded once.
 * nets_out[i] belongs to global event offsets[trial_begin] + i.
 */
int ara_oracle_event_nets(const int64_t* offsets, int64_t n_trials,
                          const uint32_t* ids, int64_t n_events,
                          const double* elts, int32_t n_pool, int64_t C,
                          int32_t J, const int32_t* elt_index,
                          const double* R, const double* Lim,
                          double occR, double occL, double aggR, double aggL,
                          int64_t trial_begin, int64_t trial_count,
                          double* nets_out, int32_t n_threads)
{
    layer_view L = {elts, C, J, elt_index, R, Lim, occR, occL};
    if (check_layer(&L, n_pool) != ORACLE_OK) return ORACLE_ERR_RANGE;
    if (trial_begin < 0 || trial_count < 0 || trial_begin + trial_count > n_trials)
        return ORACLE_ERR_ARG;
    if (offsets[n_trials] != n_events) return ORACLE_ERR_ARG;
    const int64_t first = offsets[trial_begin];
    const double A0 = apply_terms(0.0, aggR, aggL);
    int bad = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
    for (int64_t k = 0; k < trial_count; ++k) {
        int64_t t = trial_begin + k;
        exact_sum acc;
        exact_init(&acc);
        double A_prev = A0;
        for (int64_t i = offsets[t]; i < offsets[t + 1]; ++i) {
            uint32_t e = ids[i];
            if ((int64_t)e >= C) { bad |= 1; nets_out[i - first] = 0.0; continue; }
            exact_add(&acc, occurrence_loss(&L, e, NULL));
            double A = apply_terms(exact_result(&acc), aggR, aggL);
            nets_out[i - first] = A - A_prev;
            A_prev = A;
        }
    }
    return bad ? ORACLE_ERR_RANGE : ORACLE_OK;
}

/* y(E) and o(E) for every catalogue event: used to calibrate layer terms from
   quantiles and to cross-check the per-occurrence arithmetic. */
int ara_oracle_occurrence_catalogue(const double* elts, int32_t n_pool, int64_t C,
                                    int32_t J, const int32_t* elt_index,
                                    const double* R, const double* Lim,
                                    double occR, double occL,
                                    double* y_out, double* o_out)
{
    layer_view L = {elts, C, J, elt_index, R, Lim, occR, occL};
    if (check_layer(&L, n_pool) != ORACLE_OK) return ORACLE_ERR_RANGE;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < C; ++e) {
        double y;
        double o = occurrence_loss(&L, (uint32_t)e, &y);
        y_out[e] = y;
        o_out[e] = o;
    }
    return ORACLE_OK;
}

/* ---------------------------------------------------------------------- */
/* gradient counts                                                         */
/* ---------------------------------------------------------------------- */
/*
 * The year loss is piecewise linear in every term, with slopes in {-1,0,1}
 * per occurrence.  Convention at the kinks: strict subgradient -- a clamp
 * passes its input's slope only when the retention-reduced value t = v - R
 * satisfies 0 < t < L; d/dR = -1 on the same condition; d/dL = 1 iff t > L;
 * zero on equality.  For trial t the derivative of YLT_t is then an integer
 * vector over theta = [R_1..R_J, Lim_1..Lim_J, OccR, OccL, AggR, AggL]:
 *
 *   a = [0 < S - AggR < AggL]            (trial inside the aggregate band)
 *   d/dAggR = -a,  d/dAggL = [S - AggR > AggL]
 *   d/dOccR = -a * #{events: 0 < y - OccR < OccL}
 *   d/dOccL =  a * #{events: y - OccR > OccL}
 *   d/dR_j  = -a * #{events in the occurrence band with 0 < l_j - R_j < Lim_j}
 *   d/dLim_j=  a * #{events in the occurrence band with l_j - R_j > Lim_j}
 *
 * counts_out is int32 [trial_count][2J+4]; s_in holds the trials' S (as
 * produced by ara_oracle_run_layer) so the aggregate decisions use the same
 * FP64 value as the year loss.
 */
int ara_oracle_grad_counts(const int64_t* offsets, int64_t n_trials,
                           const uint32_t* ids, int64_t n_events,
                           const double* elts, int32_t n_pool, int64_t C,
                           int32_t J, const int32_t* elt_index,
                           const double* R, const double* Lim,
                           double occR, double occL, double aggR, double aggL,
                           int64_t trial_begin, int64_t trial_count,
                           const double* s_in, int32_t* counts_out, int32_t n_threads)
{
    layer_view L = {elts, C, J, elt_index, R, Lim, occR, occL};
    if (check_layer(&L, n_pool) != ORACLE_OK) return ORACLE_ERR_RANGE;
    if (trial_begin < 0 || trial_count < 0 || trial_begin + trial_count > n_trials)
        return ORACLE_ERR_ARG;
    if (offsets[n_trials] != n_events) return ORACLE_ERR_ARG;
    const int32_t P = 2 * J + 4;
    int bad = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t k = 0; k < trial_count; ++k) {
        int64_t t = trial_begin + k;
        int32_t* c = counts_out + k * P;
        for (int32_t q = 0; q < P; ++q) c[q] = 0;
        double ta = s_in[k] - aggR;
        int in_agg = (ta > 0.0) && (ta < aggL);
        int above_agg = ta > aggL;
        c[2 * J + 2] = in_agg ? -1 : 0;
        c[2 * J + 3] = above_agg ? 1 : 0;
        if (!in_agg) continue;
        for (int64_t i = offsets[t]; i < offsets[t + 1]; ++i) {
            uint32_t e = ids[i];
            if ((int64_t)e >= C) { bad |= 1; continue; }
            double y;
            (void)occurrence_loss(&L, e, &y);
            double to = y - occR;
            int in_occ = (to > 0.0) && (to < occL);
            int above_occ = to > occL;
            if (above_occ) c[2 * J + 1] += 1;
            if (!in_occ) continue;
            c[2 * J] -= 1;
            for (int32_t j = 0; j < J; ++j) {
                double l = elts[(int64_t)elt_index[j] * C + (int64_t)e];
                double tj = l - R[j];
                if (tj > 0.0 && tj < Lim[j]) c[j] -= 1;
                if (tj > Lim[j]) c[J + j] += 1;
            }
        }
    }
    return bad ? ORACLE_ERR_RANGE : ORACLE_OK;
}

int ara_oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
