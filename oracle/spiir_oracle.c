/*
 * FP64 reference for multi-rate SPIIR filtering — TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * this file.  The HIP library never calls it and shares no code with it.
 *
 * What it computes (Guo et al., "Acceleration of low-latency gravitational wave
 * searches using Maxwell-microarchitecture GPUs"):
 *
 *   every filter l of template t at band h runs the delayed first-order complex
 *   recurrence of §2.1, Eq. (7):
 *        y_l[k] = a1_l * y_l[k-1] + b0_l * x_h[k - d_l]
 *   and the band output is the sum over the template's filters, §2.1, Eq. (8),
 *   taken without the 2*dt factor (any scale is folded into b0):
 *        z_{t,h}[k] = sum_l y_l[k]
 *
 *   the multi-rate scheme of §2.2 (Fig. "multi"): the input is halved in rate
 *   band after band, x_h = D(x_{h-1}); each band is filtered with its own
 *   filters; the lowest band's output is upsampled by 2 and added to the next
 *   band's output, and so on up to the input rate.
 *
 * Readings where the paper is silent (all arithmetic is double complex):
 *   - zero state and zero input before the stream starts;
 *   - d counts samples at the band's own rate, d = 0 is the current sample;
 *   - D is a causal T_d-tap FIR that keeps even absolute indices:
 *        x_h[m] = sum_{j<T_d} h_d[j] * x_{h-1}[2m - j];
 *   - the upsample-and-add uses the zero-stuffed signal v (v[2m] = acc_{h+1}[m],
 *     v[odd] = 0) and a causal T_u-tap FIR:
 *        acc_h[k] = z_{t,h}[k] + sum_{j<T_u} h_u[j] * v[k - j],
 *     with acc_{H-1} = z_{t,H-1} and the output z_t = acc_0 (Horner order, as
 *     the text describes the chain);
 *   - the stream is processed in blocks whose length is a multiple of 2^(H-1);
 *     the block result equals the whole-stream result.
 */
#include <complex.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

typedef struct oracle_bank {
    int T, H;
    int32_t* M;       /* [T*H] filters per (template, band) */
    int64_t* moff;    /* [T*H] first filter of the segment */
    cplx* a1;         /* per filter */
    cplx* b0;
    int32_t* d;
    cplx* y;          /* per filter: state y_l[k-1] carried between blocks */
    int td, tu;
    double* hd;
    double* hu;
    int64_t done;     /* samples consumed at the base rate */
    /* full input history of every band, indexed by absolute sample */
    double** xh;
    int64_t* xh_cap;
    /* per template and band boundary: the last hu_len samples of acc_{h+1} */
    int hu_len;
    cplx* uphist;     /* [T][H-1][hu_len] */
} oracle_bank;

/* ---- the single delayed filter, Eq. (7), from a given state -------------- */

/* Runs y[k] = a1*y[k-1] + b0*x[k - d] for k in [k0, k0+n), where x is indexed by
 * absolute sample and x[i] = 0 for i < 0.  The input is xr + i*xi (xi may be
 * NULL for a real input).  y_in is y[k0-1]; the outputs are added into
 * acc[0..n).  Returns y[k0+n-1]. */
static cplx filter_run(cplx a1, cplx b0, int32_t d, const double* xr, const double* xi,
                       int64_t k0, int64_t n, cplx y_in, cplx* acc)
{
    cplx y = y_in;
    for (int64_t k = 0; k < n; ++k) {
        int64_t i = k0 + k - d;
        cplx xk = 0.0;
        if (i >= 0) xk = xi ? xr[i] + I * xi[i] : xr[i];
        y = a1 * y + b0 * xk;
        acc[k] += y;
    }
    return y;
}

/* Threads of the template loop (n <= 0: the OpenMP default); returns the count
 * the next parallel region will use.  Timing only: results do not depend on it. */
int oracle_threads(int n)
{
    static int dflt = 0;
    if (dflt == 0) dflt = omp_get_max_threads();
    omp_set_num_threads(n > 0 ? n : dflt);
    return omp_get_max_threads();
}

/* Exposed for the closed-form pins: one filter from zero state over a complex
 * input x[0..n), output y[0..n). */
void oracle_filter_one(const double* a1, const double* b0, int32_t d, const double* x_re,
                       const double* x_im, int64_t n, double* y_c)
{
    cplx a = a1[0] + I * a1[1], b = b0[0] + I * b0[1];
    cplx* y = (cplx*)calloc((size_t)(n > 0 ? n : 1), sizeof(cplx));
    filter_run(a, b, d, x_re, x_im, 0, n, 0.0, y);
    for (int64_t k = 0; k < n; ++k) { y_c[2 * k] = creal(y[k]); y_c[2 * k + 1] = cimag(y[k]); }
    free(y);
}

/* ---- resampling, §2.2 --------------------------------------------------- */

/* One /2 stage: out[m] = sum_j hd[j] * in[2m - j] for absolute m in [m0, m0+cnt);
 * `in` is indexed by absolute sample of the higher rate, zero before 0. */
static void downsample_run(const double* hd, int td, const double* in, int64_t m0, int64_t cnt,
                           double* out)
{
    for (int64_t m = 0; m < cnt; ++m) {
        double s = 0.0;
        for (int j = 0; j < td; ++j) {
            int64_t i = 2 * (m0 + m) - j;
            if (i >= 0) s += hd[j] * in[i];
        }
        out[m] = s;
    }
}

/* Exposed for the pins: a whole-signal /2 stage from zero history. */
void oracle_downsample(const double* hd, int td, const double* in, int64_t n_in, double* out)
{
    (void)n_in;
    downsample_run(hd, td, in, 0, n_in / 2, out);
}

/* One x2 upsample-and-add stage.  `ext` holds hu_len samples of the low-rate
 * signal before this block followed by its cnt/2 new samples; z is this band's
 * own output for the block (cnt samples).  acc[k] = z[k] + sum_j hu[j] v[k-j]. */
static void upsample_add_run(const double* hu, int tu, const cplx* ext, int hu_len,
                             const cplx* z, int64_t cnt, cplx* acc)
{
    for (int64_t k = 0; k < cnt; ++k) {
        cplx s = z[k];
        for (int j = 0; j < tu; ++j) {
            int64_t m = k - j;          /* index into the zero-stuffed signal v */
            if (m % 2 != 0) continue;   /* odd positions of v are the inserted zeros */
            int64_t e = hu_len + m / 2; /* position of v[m] = low[m/2] in ext */
            if (e >= 0) s += hu[j] * ext[e];
        }
        acc[k] = s;
    }
}

/* Exposed for the pins: one x2 upsample-and-add from zero history.
 * low[0..n_low), z[0..2*n_low) -> acc[0..2*n_low), complex interleaved. */
void oracle_upsample_add(const double* hu, int tu, const double* low_c, int64_t n_low,
                         const double* z_c, double* acc_c)
{
    int hl = (tu + 1) / 2;
    cplx* ext = (cplx*)calloc((size_t)(hl + n_low), sizeof(cplx));
    cplx* z = (cplx*)calloc((size_t)(2 * n_low + 1), sizeof(cplx));
    cplx* acc = (cplx*)malloc(sizeof(cplx) * (size_t)(2 * n_low + 1));
    for (int64_t m = 0; m < n_low; ++m) ext[hl + m] = low_c[2 * m] + I * low_c[2 * m + 1];
    for (int64_t k = 0; k < 2 * n_low; ++k) z[k] = z_c[2 * k] + I * z_c[2 * k + 1];
    upsample_add_run(hu, tu, ext, hl, z, 2 * n_low, acc);
    for (int64_t k = 0; k < 2 * n_low; ++k) { acc_c[2 * k] = creal(acc[k]); acc_c[2 * k + 1] = cimag(acc[k]); }
    free(ext);
    free(z);
    free(acc);
}

/* ---- the bank ----------------------------------------------------------- */

oracle_bank* oracle_create(int T, int H, const int32_t* n_filters, const double* a1_c,
                           const double* b0_c, const int32_t* delay, int td, const double* hd,
                           int tu, const double* hu)
{
    if (T < 0 || H < 1 || (H > 1 && (td < 1 || tu < 1))) return NULL;
    oracle_bank* b = (oracle_bank*)calloc(1, sizeof(oracle_bank));
    b->T = T;
    b->H = H;
    b->M = (int32_t*)malloc(sizeof(int32_t) * (size_t)(T * H + 1));
    b->moff = (int64_t*)malloc(sizeof(int64_t) * (size_t)(T * H + 1));
    int64_t nf = 0;
    for (int s = 0; s < T * H; ++s) {
        b->M[s] = n_filters[s];
        b->moff[s] = nf;
        nf += n_filters[s];
    }
    b->a1 = (cplx*)malloc(sizeof(cplx) * (size_t)(nf + 1));
    b->b0 = (cplx*)malloc(sizeof(cplx) * (size_t)(nf + 1));
    b->d = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nf + 1));
    b->y = (cplx*)calloc((size_t)(nf + 1), sizeof(cplx));
    for (int64_t l = 0; l < nf; ++l) {
        b->a1[l] = a1_c[2 * l] + I * a1_c[2 * l + 1];
        b->b0[l] = b0_c[2 * l] + I * b0_c[2 * l + 1];
        b->d[l] = delay[l];
    }
    b->td = H > 1 ? td : 0;
    b->tu = H > 1 ? tu : 0;
    b->hd = (double*)malloc(sizeof(double) * (size_t)(b->td + 1));
    b->hu = (double*)malloc(sizeof(double) * (size_t)(b->tu + 1));
    if (H > 1) {
        memcpy(b->hd, hd, sizeof(double) * (size_t)td);
        memcpy(b->hu, hu, sizeof(double) * (size_t)tu);
    }
    b->xh = (double**)calloc((size_t)H, sizeof(double*));
    b->xh_cap = (int64_t*)calloc((size_t)H, sizeof(int64_t));
    b->hu_len = (b->tu + 1) / 2;
    b->uphist = (cplx*)calloc((size_t)T * (size_t)(H - 1) * (size_t)b->hu_len + 1, sizeof(cplx));
    return b;
}

void oracle_destroy(oracle_bank* b)
{
    if (!b) return;
    for (int h = 0; h < b->H; ++h) free(b->xh[h]);
    free(b->xh);
    free(b->xh_cap);
    free(b->M);
    free(b->moff);
    free(b->a1);
    free(b->b0);
    free(b->d);
    free(b->y);
    free(b->hd);
    free(b->hu);
    free(b->uphist);
    free(b);
}

static void ensure_cap(oracle_bank* b, int h, int64_t need)
{
    if (b->xh_cap[h] >= need) return;
    int64_t cap = b->xh_cap[h] ? b->xh_cap[h] : 1024;
    while (cap < need) cap *= 2;
    b->xh[h] = (double*)realloc(b->xh[h], sizeof(double) * (size_t)cap);
    b->xh_cap[h] = cap;
}

/* Processes the next n samples (n a multiple of 2^(H-1)).  z is complex
 * interleaved, [T][n] at the base rate.  `templates_lo/hi` restrict the work to
 * a range of templates (the others' states are left untouched), which the
 * benchmark uses to time a bounded sample.  Returns 0, or -1 on a bad n. */
int oracle_process_range(oracle_bank* b, const double* x, int64_t n, double* z_c, int t_lo,
                         int t_hi)
{
    const int H = b->H;
    if (n < 0 || (n % ((int64_t)1 << (H - 1))) != 0) return -1;
    if (t_lo < 0) t_lo = 0;
    if (t_hi > b->T) t_hi = b->T;

    /* inputs of every band for this block: x_0 = x, x_h = D(x_{h-1}) */
    for (int h = 0; h < H; ++h) {
        int64_t d0 = b->done >> h, cnt = n >> h;
        ensure_cap(b, h, d0 + cnt);
        if (h == 0)
            memcpy(b->xh[0] + d0, x, sizeof(double) * (size_t)cnt);
        else
            downsample_run(b->hd, b->td, b->xh[h - 1], d0, cnt, b->xh[h] + d0);
    }

#pragma omp parallel
    {
        cplx** zb = (cplx**)malloc(sizeof(cplx*) * (size_t)H);
        for (int h = 0; h < H; ++h) zb[h] = (cplx*)malloc(sizeof(cplx) * (size_t)((n >> h) + 1));
        cplx* ext = (cplx*)malloc(sizeof(cplx) * (size_t)(n + b->hu_len + 1));
        cplx* acc = (cplx*)malloc(sizeof(cplx) * (size_t)(n + 1));

#pragma omp for schedule(dynamic, 1)
        for (int t = t_lo; t < t_hi; ++t) {
            /* every band of template t: z_{t,h} = sum over its filters */
            for (int h = 0; h < H; ++h) {
                int64_t d0 = b->done >> h, cnt = n >> h;
                for (int64_t k = 0; k < cnt; ++k) zb[h][k] = 0.0;
                int s = t * H + h;
                if (b->M[s] == 0) continue;
                for (int32_t l = 0; l < b->M[s]; ++l) {
                    int64_t f = b->moff[s] + l;
                    b->y[f] = filter_run(b->a1[f], b->b0[f], b->d[f], b->xh[h], NULL, d0, cnt,
                                         b->y[f], zb[h]);
                }
            }
            /* the upsample-and-add chain, lowest band first */
            int64_t cnt_low = n >> (H - 1);
            for (int64_t k = 0; k < cnt_low; ++k) acc[k] = zb[H - 1][k];
            for (int h = H - 2; h >= 0; --h) {
                int64_t cnt_lo = n >> (h + 1), cnt_hi = n >> h;
                cplx* hist = b->uphist + ((size_t)t * (size_t)(H - 1) + (size_t)h) * (size_t)b->hu_len;
                for (int i = 0; i < b->hu_len; ++i) ext[i] = hist[i];
                for (int64_t m = 0; m < cnt_lo; ++m) ext[b->hu_len + m] = acc[m];
                upsample_add_run(b->hu, b->tu, ext, b->hu_len, zb[h], cnt_hi, acc);
                for (int i = 0; i < b->hu_len; ++i) hist[i] = ext[cnt_lo + i];
            }
            for (int64_t k = 0; k < n; ++k) {
                z_c[2 * ((size_t)t * (size_t)n + (size_t)k)] = creal(acc[k]);
                z_c[2 * ((size_t)t * (size_t)n + (size_t)k) + 1] = cimag(acc[k]);
            }
        }
        for (int h = 0; h < H; ++h) free(zb[h]);
        free(zb);
        free(ext);
        free(acc);
    }
    b->done += n;
    return 0;
}

int oracle_process(oracle_bank* b, const double* x, int64_t n, double* z_c)
{
    return oracle_process_range(b, x, n, z_c, 0, b->T);
}

int64_t oracle_samples_done(const oracle_bank* b) { return b->done; }
