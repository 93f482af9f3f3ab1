/*
 * FP64 CPU oracle for aggregate risk analysis with secondary uncertainty
 * (Varghese & Rau-Chaplin, "Accounting for Secondary Uncertainty: Efficient
 * Computation of Portfolio Risk Measures on Multi and Many Core
 * Architectures", WHPCF'13).
 *
 * TEST INFRASTRUCTURE.  This file is a plain, slow, obviously correct
 * restatement of the method, used only by the tests, the smoke check and the
 * CPU baseline leg of the benchmark.  The product path never links, loads or
 * calls it, and it shares no code, header, table or constant generator with
 * the HIP path.
 *
 * Every step follows the paper's order:
 *   Algorithm 1 (section 2.2): for each trial, for each event of the trial,
 *     for each XELT of the layer: look up, apply secondary uncertainty, apply
 *     the XELT's financial terms, accumulate; then occurrence terms; then
 *     aggregate terms on the cumulative sum (section 2.3); one YLT value per
 *     trial (section 2.4).
 *   Section 3.2: combine the independent and correlated standard deviations
 *     in five steps (uniform -> normal -> linear combination -> normalise ->
 *     uniform).
 *   Section 3.3: moment-matched Beta parameters with the standard-deviation
 *     upper bound, and loss = max_l * InvCDF_beta(z; alpha, beta).
 *
 * Readings of points where the paper is silent or garbled (listed with the
 * reasons in the design notes of the repository):
 *   - occurrence/aggregate terms are min(max(l - R, 0), L) (the ", 0" is
 *     missing in section 2.3);
 *   - the per-event accumulator is reset per event and the aggregate terms are
 *     applied once to the trial's cumulative occurrence loss;
 *   - the per-XELT terms I are (deductible, limit, share), applied as
 *     share * min(max(l - deductible, 0), limit);
 *   - the std clamp is sigma_beta <- min(sigma_beta, c * sigma_beta_max) with
 *     c = 0.999 ("a value very close to" the bound, section 3.3);
 *   - the random numbers z_(Prog,E) and z_(E) of section 3.1 are generated,
 *     not stored: u_I = U(Philox4x32-10, key (seed, program), counter
 *     (trial, slot, elt, 0)) and u_C = U(Philox4x32-10, key (seed, ~0),
 *     counter (trial, slot, ~0, 1)), first output word, with
 *     U(w) = (2 * (w >> 9) + 1) * 2^-24;
 *   - sigma = 0 is the degenerate distribution at the mean.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, written from Salmon, Moraes, Dror & Shaw, "Parallel random   */
/* numbers: as easy as 1, 2, 3", SC'11: ten rounds of two 32x32->64 products  */
/* with a Weyl-sequence key schedule.                                         */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {                       /* key schedule between rounds */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* 32-bit word -> uniform on the open interval: odd multiples of 2^-24. */
double orc_uniform(uint32_t w)
{
    return (double)(2u * (w >> 9) + 1u) * 0x1p-24;
}

/* z_(Prog,E) of section 3.1: program- and occurrence-specific. */
double orc_u_indep(uint32_t seed, uint32_t program, uint32_t trial, uint32_t slot, uint32_t elt)
{
    uint32_t c[4] = {trial, slot, elt, 0u}, k[2] = {seed, program}, o[4];
    orc_philox4x32_10(c, k, o);
    return orc_uniform(o[0]);
}

/* z_(E) of section 3.1: occurrence-specific, shared across programs/XELTs. */
double orc_u_corr(uint32_t seed, uint32_t trial, uint32_t slot)
{
    uint32_t c[4] = {trial, slot, 0xFFFFFFFFu, 1u}, k[2] = {seed, 0xFFFFFFFFu}, o[4];
    orc_philox4x32_10(c, k, o);
    return orc_uniform(o[0]);
}

/* ------------------------------------------------------------------------- */
/* Standard normal quantile: Wichura, "Algorithm AS 241: The percentage      */
/* points of the normal distribution", Applied Statistics 37 (1988), PPND16  */
/* (rational approximations accurate to about 1e-16).                        */
/* ------------------------------------------------------------------------- */
double orc_norm_quantile(double p)
{
    if (!(p > 0.0)) return -INFINITY;
    if (!(p < 1.0)) return INFINITY;
    double q = p - 0.5;
    if (fabs(q) <= 0.425) {
        double r = 0.180625 - q * q;
        double num = ((((((2.5090809287301226727e+3 * r + 3.3430575583588128105e+4) * r
                        + 6.7265770927008700853e+4) * r + 4.5921953931549871457e+4) * r
                        + 1.3731693765509461125e+4) * r + 1.9715909503065514427e+3) * r
                        + 1.3314166789178437745e+2) * r + 3.3871328727963666080e0;
        double den = ((((((5.2264952788528545610e+3 * r + 2.8729085735721942674e+4) * r
                        + 3.9307895800092710610e+4) * r + 2.1213794301586595867e+4) * r
                        + 5.3941960214247511077e+3) * r + 6.8718700749205790830e+2) * r
                        + 4.2313330701600911252e+1) * r + 1.0;
        return q * num / den;
    }
    double r = (q < 0.0) ? p : 1.0 - p;
    r = sqrt(-log(r));
    double val;
    if (r <= 5.0) {
        r -= 1.6;
        double num = ((((((7.74545014278341407640e-4 * r + 2.27238449892691845833e-2) * r
                        + 2.41780725177450611770e-1) * r + 1.27045825245236838258e0) * r
                        + 3.64784832476320460504e0) * r + 5.76949722146069140550e0) * r
                        + 4.63033784615654529590e0) * r + 1.42343711074968357734e0;
        double den = ((((((1.05075007164441684324e-9 * r + 5.47593808499534494600e-4) * r
                        + 1.51986665636164571966e-2) * r + 1.48103976427480074590e-1) * r
                        + 6.89767334985100004550e-1) * r + 1.67638483018380384940e0) * r
                        + 2.05319162663775882187e0) * r + 1.0;
        val = num / den;
    } else {
        r -= 5.0;
        double num = ((((((2.01033439929228813265e-7 * r + 2.71155556874348757815e-5) * r
                        + 1.24266094738807843860e-3) * r + 2.65321895265761230930e-2) * r
                        + 2.96560571828504891230e-1) * r + 1.78482653991729133580e0) * r
                        + 5.46378491116411436990e0) * r + 6.65790464350110377720e0;
        double den = ((((((2.04426310338993978564e-15 * r + 1.42151175831644588870e-7) * r
                        + 1.84631831751005468180e-5) * r + 7.86869131145613259100e-4) * r
                        + 1.48753612908506148525e-2) * r + 1.36929880922735805310e-1) * r
                        + 5.99832206555887937690e-1) * r + 1.0;
        val = num / den;
    }
    return (q < 0.0) ? -val : val;
}

/* Standard normal CDF (section 3.2, fifth step): Phi(v) = erfc(-v/sqrt 2)/2. */
double orc_norm_cdf(double v)
{
    return 0.5 * erfc(-v * 0.70710678118654752440);
}

/* Section 3.2: combine sigma_I and sigma_C into one uniform z. */
double orc_combine(double u_i, double u_c, double sigma_i, double sigma_c)
{
    double sigma = sigma_i + sigma_c;               /* step 1 */
    if (sigma_c == 0.0) return u_i;                 /* the paper's two extreme cases */
    if (sigma_i == 0.0) return u_c;
    double v_p = orc_norm_quantile(u_i);            /* step 2 */
    double v_e = orc_norm_quantile(u_c);
    double wi = sigma_i / sigma, wc = sigma_c / sigma;
    double lc = v_p * wi + v_e * wc;                /* step 3 */
    double v = lc / sqrt(wi * wi + wc * wc);        /* step 4 */
    return orc_norm_cdf(v);                         /* step 5 */
}

/* ------------------------------------------------------------------------- */
/* Section 3.3: moment-matched Beta parameters.                               */
/* Returns 1 for the degenerate (sigma = 0) distribution, 0 otherwise.       */
/* ------------------------------------------------------------------------- */
int orc_beta_params(double mean, double sigma, double max_loss, double clamp_c,
                    double *alpha, double *beta, double *mu_beta)
{
    double mub = mean / max_loss;
    *mu_beta = mub;
    if (sigma == 0.0) { *alpha = 0.0; *beta = 0.0; return 1; }
    double sb = sigma / max_loss;
    double sbmax = sqrt(mub * (1.0 - mub));
    if (sb > clamp_c * sbmax) sb = clamp_c * sbmax;
    double nu = (sbmax / sb) * (sbmax / sb) - 1.0;
    *alpha = mub * nu;
    *beta = (1.0 - mub) * nu;
    return 0;
}

/* ln B(a,b) from its definition through the gamma function.  Extended
 * precision keeps lgamma(b) - lgamma(a+b) from cancelling when a << b. */
static long double log_beta_l(double a, double b)
{
    return lgammal((long double)a) + lgammal((long double)b) - lgammal((long double)a + (long double)b);
}

double orc_log_beta(double a, double b)
{
    return (double)log_beta_l(a, b);
}

/* x^a (1-x)^b / B(a,b), the factor in front of the continued fraction. */
static double beta_front(double x, double a, double b, long double lnB)
{
    long double e = (long double)a * logl((long double)x) + (long double)b * log1pl(-(long double)x) - lnB;
    return (double)expl(e);
}

/* ------------------------------------------------------------------------- */
/* Regularised incomplete beta I_x(a,b) = B(x;a,b)/B(a,b) (section 3.3).      */
/* Continued fraction (DLMF 8.17.22), evaluated with the modified Lentz      */
/* method; the fraction converges fast for x < (a+1)/(a+b+2), and the        */
/* reflection I_x(a,b) = 1 - I_{1-x}(b,a) covers the other side.             */
/* ------------------------------------------------------------------------- */
static double cf_value(double x, double a, double b)
{
    /* returns 1/(1 + d1/(1 + d2/(1 + ...))) */
    const double tiny = 1e-300;
    double f = 1.0, C = 1.0, D = 0.0;
    for (int n = 1; n <= 20000; ++n) {
        int m = n / 2;
        double d;
        if (n & 1)
            d = -(a + m) * (a + b + m) * x / ((a + 2.0 * m) * (a + 2.0 * m + 1.0));
        else
            d = m * (b - m) * x / ((a + 2.0 * m - 1.0) * (a + 2.0 * m));
        D = 1.0 + d * D;
        if (fabs(D) < tiny) D = tiny;
        C = 1.0 + d / C;
        if (fabs(C) < tiny) C = tiny;
        D = 1.0 / D;
        double delta = C * D;
        f *= delta;
        if (fabs(delta - 1.0) < 1e-16) break;
    }
    return 1.0 / f;
}

/* I_x(a,b) - u, arranged so that neither tail loses digits to cancellation. */
static double cdf_minus(double x, double a, double b, long double lnB, double u)
{
    if (x <= 0.0) return -u;
    if (x >= 1.0) return 1.0 - u;
    double front = beta_front(x, a, b, lnB);
    if (x <= (a + 1.0) / (a + b + 2.0))
        return front / a * cf_value(x, a, b) - u;
    double upper = front / b * cf_value(1.0 - x, b, a);    /* = 1 - I_x(a,b) */
    return (1.0 - u) - upper;
}

double orc_beta_inc(double x, double a, double b)
{
    if (x <= 0.0) return 0.0;
    if (x >= 1.0) return 1.0;
    return cdf_minus(x, a, b, log_beta_l(a, b), 0.0);
}

/* Beta density, the derivative used by Newton's method. */
static double beta_pdf(double x, double a, double b, long double lnB)
{
    return beta_front(x, a, b, lnB) / (x * (1.0 - x));
}

static uint64_t dbits(double x) { uint64_t u; memcpy(&u, &x, 8); return u; }
static double bitsd(uint64_t u) { double x; memcpy(&x, &u, 8); return x; }

/*
 * Inverse of the regularised incomplete beta (section 3.3): the smallest
 * double x in [0,1] with I_x(a,b) >= u.  The CDF is strictly increasing, so
 * the root is unique.  The root is kept in a bracket [lo, hi] of doubles,
 * stored as IEEE bit patterns (monotone for non-negative doubles), so that a
 * bisection step halves the number of doubles in the bracket and at most 62
 * such steps reach adjacent doubles whatever the magnitude of the root.
 * Mode 0 takes Newton steps while they stay inside the bracket and shrink
 * geometrically, bisecting otherwise; mode 1 bisects only (cross-check).
 */
double orc_beta_inc_inv(double u, double a, double b, int pure_bisection, int *n_iter)
{
    int it = 0;
    if (n_iter) *n_iter = 0;
    if (u <= 0.0) return 0.0;
    if (u >= 1.0) return 1.0;
    long double lnB = log_beta_l(a, b);
    uint64_t lo = dbits(0.0), hi = dbits(1.0);       /* F(lo) < u <= F(hi) */
    double x = pure_bisection ? bitsd(lo + (hi - lo) / 2) : a / (a + b);
    double prev_step = INFINITY;
    for (it = 1; it <= 1000; ++it) {
        double g = cdf_minus(x, a, b, lnB, u);
        uint64_t xb = dbits(x);
        if (g < 0.0) lo = xb; else hi = xb;
        if (hi - lo <= 1) break;
        int bisect = pure_bisection;
        double xn = x;
        if (!bisect) {
            double p = beta_pdf(x, a, b, lnB);
            double step = g / p;
            xn = x - step;
            if (!(p > 0.0) || !(xn > bitsd(lo) && xn < bitsd(hi)) || !(fabs(step) <= 0.5 * prev_step)) {
                bisect = 1;
                prev_step = INFINITY;
            } else {
                prev_step = fabs(step);
                if (fabs(step) <= 0x1p-53 * xn) { x = xn; break; }   /* converged to rounding */
            }
        }
        if (bisect) xn = bitsd(lo + (hi - lo) / 2);
        x = xn;
    }
    if (n_iter) *n_iter = it;
    if (hi - lo <= 1) return bitsd(hi);
    return x;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 1 for one layer over a set of trials.                            */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t n;
    const int32_t *event_id;
    const double *mean, *sigma_i, *sigma_c;   /* sigma_c may be NULL (= 0) */
    const double *max_loss;
    double deductible, limit, share;          /* per-XELT financial terms I */
} orc_elt;

typedef struct {
    double occ_retention, occ_limit, agg_retention, agg_limit;
} orc_layer_terms;

enum { ORC_MODE_MEAN = 0, ORC_MODE_PLAIN = 1 };

static double clamp_xl(double l, double retention, double limit)
{
    double v = l - retention;
    if (v < 0.0) v = 0.0;
    return v < limit ? v : limit;
}

/*
 * yet_rows: [n_rows][K] event IDs of the selected trials; trial_ids: their
 * trial numbers (the RNG counter).  Outputs per selected trial: ylt (the
 * trial's year loss), gross (sum of share * loss over all draws, the scale of
 * the GPU tolerance) and max_occ (the largest occurrence loss net of
 * occurrence terms).  yelt (optional, n_rows x K) receives each event
 * occurrence's loss net of XELT and occurrence terms, the quantity the
 * aggregate terms are applied to the sum of (section 2.4's per-occurrence
 * view).  Returns 0, or -1 for an event ID outside the catalog.
 */
int orc_run_layer(const int32_t *yet_rows, const int64_t *trial_ids, int64_t n_rows,
                  int32_t K, int32_t C, const orc_elt *elts, int32_t n_elts,
                  const orc_layer_terms *lt, uint32_t seed, uint32_t program_id,
                  int32_t mode, double clamp_c, double *ylt, double *gross,
                  double *max_occ, double *yelt, int32_t n_threads)
{
    /* Stage 1 (section 2.2, preprocessing): direct-access tables, one per
     * XELT, indexed by event ID over the catalog (section 4.1). */
    int32_t **table = (int32_t **)calloc((size_t)n_elts, sizeof(int32_t *));
    double **alpha = (double **)calloc((size_t)n_elts, sizeof(double *));
    double **beta = (double **)calloc((size_t)n_elts, sizeof(double *));
    double **mub = (double **)calloc((size_t)n_elts, sizeof(double *));
    int rc = 0;
    for (int j = 0; j < n_elts; ++j) {
        table[j] = (int32_t *)malloc((size_t)C * sizeof(int32_t));
        for (int32_t e = 0; e < C; ++e) table[j][e] = -1;
        alpha[j] = (double *)malloc((size_t)elts[j].n * sizeof(double));
        beta[j] = (double *)malloc((size_t)elts[j].n * sizeof(double));
        mub[j] = (double *)malloc((size_t)elts[j].n * sizeof(double));
        for (int32_t r = 0; r < elts[j].n; ++r) {
            table[j][elts[j].event_id[r]] = r;
            double sc = elts[j].sigma_c ? elts[j].sigma_c[r] : 0.0;
            orc_beta_params(elts[j].mean[r], elts[j].sigma_i[r] + sc, elts[j].max_loss[r],
                            clamp_c, &alpha[j][r], &beta[j][r], &mub[j][r]);
        }
    }

    /* Stage 2: the simulation, one trial per OpenMP iteration (trials are
     * independent, section 4.3). */
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (int64_t r = 0; r < n_rows; ++r) {
        uint32_t trial = (uint32_t)trial_ids[r];
        const int32_t *row = yet_rows + r * (int64_t)K;
        double S = 0.0, Scomp = 0.0, G = 0.0, omax = 0.0;
        for (int32_t k = 0; k < K; ++k) {                 /* each event E in T */
            int32_t e = row[k];
            if (e < 0 || e >= C) { rc = -1; continue; }
            double lT = 0.0;                              /* per-event accumulator */
            for (int32_t j = 0; j < n_elts; ++j) {        /* each XELT covered by L */
                int32_t idx = table[j][e];                /* lookup l_E */
                if (idx < 0) continue;                    /* zero loss: nothing to draw */
                const orc_elt *X = &elts[j];
                double loss;
                if (mode == ORC_MODE_MEAN) {
                    loss = X->mean[idx];
                } else {                                  /* apply secondary uncertainty */
                    double si = X->sigma_i[idx];
                    double sc = X->sigma_c ? X->sigma_c[idx] : 0.0;
                    if (si + sc == 0.0) {
                        loss = X->mean[idx];
                    } else {
                        double ui = orc_u_indep(seed, program_id, trial, (uint32_t)k, (uint32_t)j);
                        double uc = (sc > 0.0) ? orc_u_corr(seed, trial, (uint32_t)k) : 0.5;
                        double z = orc_combine(ui, uc, si, sc);
                        double x = orc_beta_inc_inv(z, alpha[j][idx], beta[j][idx], 0, NULL);
                        loss = X->max_loss[idx] * x;
                    }
                }
                G += X->share * loss;
                lT += X->share * clamp_xl(loss, X->deductible, X->limit);   /* terms I */
            }
            double o = clamp_xl(lT, lt->occ_retention, lt->occ_limit);     /* occurrence terms */
            if (yelt) yelt[r * (int64_t)K + k] = o;
            if (o > omax) omax = o;
            double t = S + o;                             /* Neumaier-compensated sum */
            if (fabs(S) >= fabs(o)) Scomp += (S - t) + o; else Scomp += (o - t) + S;
            S = t;
        }
        S += Scomp;
        ylt[r] = clamp_xl(S, lt->agg_retention, lt->agg_limit);           /* aggregate terms */
        if (gross) gross[r] = G;
        if (max_occ) max_occ[r] = omax;
    }

    for (int j = 0; j < n_elts; ++j) { free(table[j]); free(alpha[j]); free(beta[j]); free(mub[j]); }
    free(table); free(alpha); free(beta); free(mub);
    return rc;
}

/* Beta quantile for a vector of (u, a, b): used by the tests and to label
 * reference points for the sampling surrogate. */
void orc_beta_inc_inv_vec(const double *u, const double *a, const double *b, int64_t n,
                          int32_t pure_bisection, double *x_out, int32_t n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n; ++i)
        x_out[i] = orc_beta_inc_inv(u[i], a[i], b[i], pure_bisection, NULL);
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
