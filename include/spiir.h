/*
 * spiir.h — C ABI of the MI355X SPIIR filtering library (libspiir.so).
 *
 * The library runs Summed Parallel IIR (SPIIR) filtering, single-rate and
 * multi-rate, on one AMD Instinct MI355X (gfx950) with hand-written HIP kernels.
 * It follows Guo et al., "Acceleration of low-latency gravitational wave
 * searches using Maxwell-microarchitecture GPUs":
 *
 *   §2.1, Eq. (7):  every filter l of a template runs the delayed first-order
 *                   complex recurrence  y_l[k] = a1_l y_l[k-1] + b0_l x[k - d_l];
 *   §2.1, Eq. (8):  the template output is the sum over its filters,
 *                   z[k] = sum_l y_l[k]  (the 2*dt factor of Eq. 8 is not
 *                   applied: fold any scale into b0; the map is linear);
 *   §2.2 (Fig. "multi"): the input is halved in rate band by band with a
 *                   low-pass FIR (Eq. 9 describes the resampling filter), each
 *                   band is filtered with its own filters, and the lowest
 *                   band's output is upsampled by 2 and added to the next
 *                   band's output, up to the input rate.
 *
 * Conventions that the paper leaves open and this library fixes:
 *   - zero filter state and zero input before the stream starts;
 *   - delays d are integer samples at the band's own rate (d = 0: current);
 *   - downsampling: x_h[m] = sum_{j<T_d} h_down[j] x_{h-1}[2m - j] (causal,
 *     keeps even absolute indices, no group-delay compensation);
 *   - upsample-and-add: acc_h[k] = z_h[k] + sum_{j<T_u} h_up[j] v[k - j], where
 *     v[2m] = acc_{h+1}[m] and v[odd] = 0; acc_{H-1} = z_{H-1}; output acc_0.
 *
 * Threading: a bank must not be used by two host threads at once; different
 * banks may be.  No call throws; every call returns a status code.
 * Memory: all device memory a bank needs is allocated by spiir_create and freed
 * by spiir_destroy; the processing calls allocate nothing.
 */
#ifndef SPIIR_H
#define SPIIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Interleaved complex64 output sample. */
typedef struct {
    float re;
    float im;
} spiir_c32;

typedef struct spiir_bank spiir_bank;

/* Status codes (0 = success, negative = error). */
enum {
    SPIIR_OK = 0,
    SPIIR_EINVAL = -1,     /* bad argument; nothing was enqueued, state unchanged   */
    SPIIR_ENOMEM = -2,     /* device allocation failed or over the stated budget    */
    SPIIR_EDEVICE = -3,    /* HIP error; the bank is poisoned and must be destroyed */
    SPIIR_EORDER = -4,     /* request order/aliasing violated (e.g. a bank twice)   */
    SPIIR_ENONFINITE = -5  /* a template's state or output became non-finite        */
};

/* Arithmetic of the filter sum. */
enum {
    SPIIR_FP32 = 0,             /* complex FP32, plain summation over filters      */
    SPIIR_FP32_COMPENSATED = 1  /* complex FP32 filters, cross-lane sums in FP64   */
};

/*
 * Bank descriptor (read only during the call that receives it; the caller
 * keeps ownership of every array).
 *
 *   n_templates, n_bands  T >= 1 templates, H in [1, 12] bands; band h runs at
 *                         base_rate_hz / 2^h.
 *   n_filters             [T*H] filters of template t at band h, index t*H + h;
 *                         0 = band inactive for that template.
 *   a1, b0                complex128 interleaved (re, im), one pair per filter,
 *                         concatenated in (template, band, filter) order; |a1|
 *                         must be < 1 for a stable filter (not enforced), all
 *                         values finite.
 *   delay                 one int32 per filter, in [0, SPIIR_MAX_DELAY], in
 *                         samples at the band's rate.
 *   n_taps_down, h_down   T_d real taps of the /2 anti-alias FIR (H > 1).
 *   n_taps_up, h_up       T_u real taps of the x2 interpolation FIR (H > 1).
 *   max_block             largest block, in base-rate samples, that
 *                         process calls will pass; a multiple of 2^(H-1).
 *   precision             SPIIR_FP32 or SPIIR_FP32_COMPENSATED.
 *   carry_chunk           C: every C samples (absolute band index) the FP32
 *                         state is corrected by (a1^C - fl32(a1)^C) times the
 *                         state at the chunk start, computed in FP64 at
 *                         create; a power of two in [16, 1024]; 0 = 32.
 *   filters_per_lane      F in {1, 2, 4, 6, 8}; 0 = library default.  With
 *                         both this and waves_per_group 0 the library takes
 *                         F = 4 with 8 waves for banks that fill the device
 *                         with such workgroups (multi-rate banks: with at
 *                         least 4 rounds of them), and F = 4 with 4 waves
 *                         otherwise.
 *   waves_per_group       wave64s per workgroup in [1, 16] ([1, 8] when
 *                         filters_per_lane is 8); 0 = default (as above;
 *                         with F given: 8, or 4 with 6 or more filters per
 *                         lane; fewer when a long delay window would not
 *                         fit the LDS).
 *   device                HIP device ordinal the bank lives on.
 *   time_chunks           P in {0, 1, 2, 4, ..., 64}; 0 or 1 = off;
 *                         SPIIR_TIME_CHUNKS_AUTO: the library picks P for
 *                         blocks of max_block samples, splitting while the
 *                         longest workgroup's run of dependent samples, cut
 *                         in P, is no shorter than the bank's filter work
 *                         per workgroup slot of the device (spiir_plan
 *                         reports the choice; P = 1 for banks that fill the
 *                         device, up to 64 for a single small template).  With
 *                         P > 1 each block is also split in time, so banks
 *                         too small to fill the device finish sooner: every
 *                         band's samples are cut at absolute multiples of a
 *                         chunk length (a multiple of C, about the block /
 *                         P); an end-state pass runs all chunks but the last
 *                         at once from zero state, a chain pass turns those
 *                         end states into each chunk's start state with
 *                         a1^length (computed in FP64 at create), and the
 *                         filter pass runs every chunk from its start state.
 *                         Results differ from P = 1 by rounding only (the
 *                         bitwise block-split invariance holds for P <= 1).
 *   window_copies         1 or 2; 0 = chosen by the library.  The filter
 *                         kernel keeps each band's input window in LDS, as
 *                         two copies shifted by one sample (each filter reads
 *                         a sample pair with one aligned 64-bit access) or as
 *                         one (two 32-bit accesses, half the LDS, so long
 *                         delay windows leave room for more workgroups per
 *                         compute unit).  The two layouts place the filters
 *                         on lanes by different LDS bank classes, so their
 *                         results differ by the order of the FP32 sum over
 *                         filters only.
 *   workspace             SPIIR_WORKSPACE_OWN (0): spiir_create allocates the
 *                         bank's workspace (the per-piece band outputs that
 *                         the filter kernel hands to the upsample-and-add
 *                         kernel within one launch sequence).
 *                         SPIIR_WORKSPACE_CALLER (1): it does not; every
 *                         request on the bank must then bring a workspace
 *                         (spiir_request.ws_dev), and the footprint leaves
 *                         it out.  The workspace holds nothing between launch
 *                         sequences, so a caller can keep a few of them for
 *                         many banks (one per launch sequence in flight)
 *                         instead of one per bank.  Results do not depend on
 *                         where the workspace lives.
 *   engine                SPIIR_ENGINE_VALU (0): the filter bank runs Eq. 7
 *                         sample by sample on the vector units.
 *                         SPIIR_ENGINE_MFMA (1), a prototype for single-rate
 *                         banks (H = 1) with the plain sum (SPIIR_FP32): the
 *                         block is cut into chunks of 8 samples at absolute
 *                         multiples of 8; the vector units carry each filter's
 *                         state from chunk to chunk (Eq. 6 applied over a chunk,
 *                         with the carry correction every C samples), and
 *                         both parts of the output inside a chunk, the carried
 *                         state times a1^(t+1) and the chunk's own inputs
 *                         times b0 a1^(t-s) (a Toeplitz matrix), are summed
 *                         over filters by fp16 matrix-core products with each
 *                         operand split into a high and a low fp16 part and
 *                         FP32 accumulation.  Requires max_block and every
 *                         block length to be multiples of 128, time_chunks
 *                         <= 1 (SPIIR_EINVAL otherwise), and filter states
 *                         below 128 in magnitude (the fp16 state operand
 *                         saturates beyond; the bank's status reports it).
 */
typedef struct {
    int32_t n_templates;
    int32_t n_bands;
    int32_t base_rate_hz;
    const int32_t* n_filters;
    const double* a1;
    const double* b0;
    const int32_t* delay;
    int32_t n_taps_down;
    const double* h_down;
    int32_t n_taps_up;
    const double* h_up;
    int32_t max_block;
    int32_t precision;
    int32_t carry_chunk;
    int32_t filters_per_lane;
    int32_t waves_per_group;
    int32_t device;
    int32_t time_chunks;
    int32_t window_copies;
    int32_t workspace;
    int32_t engine;
} spiir_bank_desc;

#define SPIIR_MAX_BANDS 12
#define SPIIR_MAX_DELAY 16383
#define SPIIR_MAX_TAPS 1024
#define SPIIR_MAX_BATCH 16
#define SPIIR_TIME_CHUNKS_AUTO (-1)
#define SPIIR_WORKSPACE_OWN 0
#define SPIIR_WORKSPACE_CALLER 1
#define SPIIR_ENGINE_VALU 0
#define SPIIR_ENGINE_MFMA 1

/*
 * One request of a batch: the next n samples of the stream bound to `bank`.
 *   ws_dev  device workspace for this request, or NULL for the bank's own
 *           (SPIIR_EINVAL if the bank has none).  At least the bank's
 *           spiir_plan_info.workspace_bytes, 256-byte aligned, caller-owned;
 *           no other request or launch sequence may use it until this one's
 *           work has completed (reuse in stream order is fine).  Its contents
 *           before and after the call do not matter.
 */
typedef struct {
    spiir_bank* bank;
    const float* x_dev;
    int64_t n;
    spiir_c32* z_dev;
    int64_t ldz;
    void* ws_dev;
} spiir_request;

/*
 * spiir_footprint — device bytes spiir_create would allocate for `desc`.
 * Pure host function: no device call, no allocation.  Returns SPIIR_EINVAL for
 * a descriptor spiir_create would reject.  Used for admission by HBM footprint.
 */
int spiir_footprint(const spiir_bank_desc* desc, size_t* bytes);

/*
 * spiir_create — validate, plan and upload a bank.
 * Copies the tables (converted to FP32 in the library's lane order), computes
 * the FP64 carry corrections on the device, and allocates state, input
 * histories, workspace and per-template up-chain histories.  `hip_stream`
 * (hipStream_t or NULL for the null stream) orders the uploads.  On success
 * *out owns all device memory; on error *out is NULL and the return is
 * SPIIR_EINVAL, SPIIR_ENOMEM or SPIIR_EDEVICE.  One bank is bound to one input
 * stream (its histories carry that stream).
 */
int spiir_create(const spiir_bank_desc* desc, void* hip_stream, spiir_bank** out);

/*
 * spiir_clone — a new bank with the tables, launch plan and workspace mode of
 * `src` (its own device copy of every table) and zero state, bound to a
 * stream of its own; as if spiir_create had been called again with src's
 * descriptor, without planning again or reading host tables.  For serving
 * one template bank on several detector streams (the paper's search runs
 * the same bank per detector, §5).  Waits for src's outstanding work; src is
 * not changed.  Same error codes as spiir_create (*out NULL on error).
 */
int spiir_clone(const spiir_bank* src, void* hip_stream, spiir_bank** out);

/*
 * spiir_process_block — filter the next n samples of the bank's stream
 * (Eqs. 7-8, and the §2.2 chain when H > 1).
 *   x_dev  device pointer, n FP32 samples at the base rate (caller-owned).
 *   n      0 < n <= max_block and n % 2^(H-1) == 0, else SPIIR_EINVAL with
 *          nothing enqueued and the state unchanged.
 *   z_dev  device pointer, complex64, row t at z_dev + t*ldz, n samples:
 *          z_dev[t*ldz + k] is the output for absolute sample
 *          (samples_done + k).  ldz >= n.
 * Asynchronous on `hip_stream`; the stream first waits for the bank's previous
 * work, so per-bank order holds across streams.  Buffers must stay valid until
 * the work completes.  Allocates nothing.
 */
int spiir_process_block(spiir_bank* bank, const float* x_dev, int64_t n, spiir_c32* z_dev,
                        int64_t ldz, void* hip_stream);

/*
 * spiir_process_block_noalloc — spiir_process_block for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same arguments, results and errors,
 * bit for bit, but the workspace of the launch sequence is a static device
 * array of SPIIR_NOALLOC_MAX_WORKSPACE bytes that the library holds on each
 * GPU it runs on until the process ends, and the call itself allocates
 * nothing (no hipMalloc, hipFree or event creation; kernel timing by
 * spiir_profile_* does not cover it).  Works for banks of either workspace
 * mode.  A bank whose workspace (spiir_plan_info.workspace_bytes) exceeds
 * the array returns SPIIR_ENOMEM with nothing enqueued.  Every call on one
 * GPU shares that GPU's array: calls whose work overlaps on the device (two
 * streams, or two host threads) race and give wrong results; calls in one
 * stream's order are safe.
 */
#define SPIIR_NOALLOC_MAX_WORKSPACE (32u << 20)
int spiir_process_block_noalloc(spiir_bank* bank, const float* x_dev, int64_t n, spiir_c32* z_dev,
                                int64_t ldz, void* hip_stream);

/*
 * spiir_process_batch — one launch sequence over up to SPIIR_MAX_BATCH
 * requests of different banks (each bank at most once: SPIIR_EORDER
 * otherwise; concatenate consecutive blocks of one stream instead).  Banks in
 * one batch must share the device (SPIIR_EINVAL otherwise); banks of
 * different launch shapes (filters per lane, lanes per group, precision) get
 * one filter launch per shape between the shared staging and up-add
 * launches.  Every result equals what separate spiir_process_block calls
 * give, bit for bit.  Validation is all-or-nothing.
 */
int spiir_process_batch(int32_t n_req, const spiir_request* req, void* hip_stream);

/*
 * Trigger reduction (the step after the filter in a search: find where |z|
 * peaks in each template's block, §5).  For every template t the block's
 * outputs z_t[k], k < n, are reduced to:
 *   peak2    max_k |z_t[k]|^2, computed from the FP32 output as re*re + im*im
 *            with each product and the sum rounded to FP32 (no FMA), so the
 *            caller can repeat every comparison exactly;
 *   index    the smallest k attaining peak2 (-1 if every |z|^2 is NaN);
 *   n_above  the number of k with |z_t[k]|^2 >= threshold*threshold (the
 *            square rounded to FP32).
 */
typedef struct {
    float peak2;
    int32_t index;
    int32_t n_above;
    int32_t reserved; /* 0 */
} spiir_peak;

/*
 * spiir_process_peaks — spiir_process_block plus the trigger reduction.
 *   z_dev     as for spiir_process_block, or NULL to skip writing z (the
 *             reduction still sees every output); ldz is ignored then.
 *   peak_dev  device array of n_templates spiir_peak (caller-owned),
 *             overwritten.
 *   threshold finite, >= 0 (SPIIR_EINVAL otherwise).
 * Results for z and the state are identical to spiir_process_block.
 */
int spiir_process_peaks(spiir_bank* bank, const float* x_dev, int64_t n, spiir_c32* z_dev,
                        int64_t ldz, spiir_peak* peak_dev, float threshold, void* hip_stream);

/*
 * spiir_process_batch_peaks — spiir_process_batch plus the trigger
 * reduction: peak_dev[r] is the spiir_peak array of request r (z_dev of a
 * request may be NULL, as above).  Same batching rules and guarantees.
 */
int spiir_process_batch_peaks(int32_t n_req, const spiir_request* req, spiir_peak* const* peak_dev,
                              float threshold, void* hip_stream);

/*
 * Recorded batches: one launch sequence, recorded once as a HIP graph and
 * replayed for every block (for loops that would otherwise pay the host cost
 * of building and launching the sequence per block).
 *
 * spiir_graph_create — record what spiir_process_batch(n_req, req) enqueues
 * (same validation and error codes) without running it and without changing
 * any bank.  The graph keeps the request's pointers and sizes: x_dev, n,
 * z_dev and ldz are fixed for its lifetime.  Allocates host and device memory
 * for the graph; returns SPIIR_EDEVICE if recording fails.
 *
 * spiir_graph_launch — replay on `hip_stream`.  Each bank of the graph takes
 * its next n samples from x_dev and writes z_dev exactly as
 * spiir_process_batch would at that point of its stream (bit for bit), and its
 * sample count advances by n; the stream first waits for the banks' previous
 * work.  The caller refills x_dev and reads z_dev between replays, in stream
 * order.  Replays and eager calls may be interleaved on a bank.
 *
 * spiir_graph_destroy — wait for the graph's last replay, free it.  It does
 * not touch the banks, so it may follow their destruction; replaying a graph
 * after one of its banks was destroyed is undefined.  NULL is accepted.
 */
typedef struct spiir_graph spiir_graph;
int spiir_graph_create(int32_t n_req, const spiir_request* req, spiir_graph** out);
int spiir_graph_launch(spiir_graph* graph, void* hip_stream);
int spiir_graph_destroy(spiir_graph* graph);

/* spiir_reset — zero every state (filters, histories, flags, sample count).
 * Synchronous. */
int spiir_reset(spiir_bank* bank);

/* spiir_state_size — bytes of the blob spiir_save_state writes. */
int spiir_state_size(const spiir_bank* bank, size_t* bytes);

/* spiir_save_state — copy the carried state (filter states, pending carry
 * corrections, input histories, up-chain histories, flags, sample count) into
 * host_buf (spiir_state_size bytes).  Waits for the bank's work. */
int spiir_save_state(spiir_bank* bank, void* host_buf, void* hip_stream);

/* spiir_load_state — restore a blob from spiir_save_state of a bank with the
 * same shape and filter layout: the same sizes, launch shape and delays, as a
 * bank created from the same descriptor has.  The blob's header carries a
 * fingerprint of the layout; SPIIR_EINVAL (state unchanged) if the header does
 * not match.  Synchronous. */
int spiir_load_state(spiir_bank* bank, const void* host_buf, void* hip_stream);

/* spiir_status — sticky non-finite flags.  Waits for the bank's work.
 * template_flags (may be NULL): host array of n_templates, set to 1 where the
 * template's state went non-finite.  Returns SPIIR_ENONFINITE if any is set,
 * SPIIR_EDEVICE if the bank is poisoned, else SPIIR_OK.  spiir_reset clears. */
int spiir_status(spiir_bank* bank, int32_t* template_flags);

/* spiir_destroy — wait for the bank's outstanding work, then free it.
 * NULL is accepted. */
int spiir_destroy(spiir_bank* bank);

/* spiir_strerror — static description of a status code. */
const char* spiir_strerror(int status);

/* ---- introspection (no effect on results) ---------------------------- */

/* Samples consumed so far, at the base rate. */
int spiir_samples_done(const spiir_bank* bank, int64_t* samples);

/* Plan summary for a descriptor, computed on the host without a device. */
typedef struct {
    int64_t total_filters;    /* sum of n_filters                              */
    int64_t filter_slots;     /* lanes x F over all workgroups (incl. padding) */
    int32_t n_groups;         /* workgroups of the filter kernel               */
    int32_t n_pieces;         /* (template, band) pieces after splitting       */
    int32_t lanes_per_group;  /* 64 x waves_per_group                          */
    int32_t filters_per_lane; /* F                                             */
    int32_t lds_bytes;        /* dynamic LDS of the filter kernel              */
    int32_t carry_chunk;      /* C                                             */
    size_t footprint;         /* device bytes spiir_create allocates           */
    int32_t time_chunks;      /* P (1 = no time split)                         */
    int32_t window_copies;    /* LDS copies of the input window (1 or 2)       */
    size_t workspace_bytes;   /* device workspace one request needs            */
    int32_t workspace;        /* SPIIR_WORKSPACE_OWN or SPIIR_WORKSPACE_CALLER */
    int32_t engine;           /* SPIIR_ENGINE_VALU or SPIIR_ENGINE_MFMA        */
} spiir_plan_info;

int spiir_plan(const spiir_bank_desc* desc, spiir_plan_info* info);

/* The same summary for a created bank (the plan spiir_create made, without
 * planning again).  SPIIR_EINVAL for NULL arguments. */
int spiir_bank_plan(const spiir_bank* bank, spiir_plan_info* info);

/* Process-wide kernel timing with HIP events recorded around each kernel the
 * library launches.  spiir_profile_enable(1) clears and starts recording;
 * spiir_profile_read waits for the recorded events and returns, per kernel
 * kind (0 = input staging and downsample cascade, 1 = filter bank, 2 =
 * upsample-and-add / output), the launch count and total milliseconds. */
typedef struct {
    int64_t launches[3];
    double ms[3];
} spiir_profile_data;

int spiir_profile_enable(int enable);
int spiir_profile_read(spiir_profile_data* out);

#ifdef __cplusplus
}
#endif

#endif /* SPIIR_H */
