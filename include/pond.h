/*
 * pond.h -- C ABI of the MI355X coherent-dedispersion + fold library.
 *
 * The operation is the pulsar mode of PONDER (Naidu, Joshi, Manoharan &
 * Krishnakumar, arXiv:1503.01405): overlap-save coherent dedispersion of
 * complex baseband voltages (Sec. 3.7, Eq. (4)), square-law detection,
 * integration of the detected series (Sec. 4: from the 62.5 ns base
 * resolution to 1 us) and folding at the pulsar period into profile bins
 * (Sec. 3.4.1 and Sec. 3.7: the fold thread writes profiles periodically).
 *
 * Conventions shared by every entry point
 *   - Frequencies are in MHz, DM in pc cm^-3, times in seconds (Sec. 3.7).
 *   - bw_mhz is the complex bandwidth, equal to the complex sample rate in
 *     Msps; baseband frequency f maps to sky frequency f0 + f.
 *   - Input is single-polarisation complex int8: I then Q per sample,
 *     interleaved, in DEVICE memory, 2-byte aligned (the real two-channel
 *     input of the pond_real_* calls is described with them).
 *   - Block b of the stream covers input samples [b*hop, b*hop + nfft).
 *     Its kept outputs are outputs m = b*hop + j, j in [0, hop); output m
 *     is input sample m + n_front, referred to arrival at f0.  Only fully
 *     covered blocks produce outputs.
 *   - Each spectrum bin k (frequency f_k = k*bw/nfft, k >= nfft/2 taken as
 *     k - nfft) is multiplied by exp(-2 pi i turns_k) with
 *     turns_k = dm f_k^2 / (2.41e-10 f0^2 (f0 + f_k)), the inverse of the
 *     ISM response of Eq. (4) with the dispersion constant of Eq. (1).
 *     The phase is evaluated and reduced mod 1 turn in float64.
 *   - Forward transform unnormalised, inverse with 1/nfft; unit taper
 *     unless one is set with pond_plan_set_taper.
 *   - Fold: x = (m + n_front) * inv_pfs with inv_pfs = 1/(period_s * fs),
 *     bin = min(floor((x - floor(x)) * nbins), nbins - 1), in float64.
 *     Sub-integration s holds outputs m in [s*S, (s+1)*S) for S =
 *     subint_nsamp (> 0), or every output (S = 0).  A profile is the mean
 *     detected power per bin (0 for an empty bin).
 *   - Calls are asynchronous on hip_stream (a hipStream_t; NULL is the
 *     null stream) and never synchronise it; all counts are derived on the
 *     host from the plan's own state.  Device pointers must stay valid, and
 *     iq unmodified, until the stream has passed the call.
 *   - A plan owns its device workspace (allocated in create, freed in
 *     destroy) and its stream state.  A plan is not thread-safe; distinct
 *     plans are independent.  Successive calls on one plan must be ordered
 *     on the device: use one stream per plan, or order the streams.  The
 *     plan is bound to the device that is current when it is created.
 *   - No entry point prints, throws or aborts.
 */
#ifndef POND_H
#define POND_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pond_plan pond_plan;

/* Return codes (negative = error). */
#define POND_OK        0
#define POND_EINVAL   (-1)  /* bad argument or call sequence; plan state untouched   */
#define POND_ENOMEM   (-2)  /* device allocation failed; plan state untouched        */
#define POND_EDEVICE  (-3)  /* HIP runtime error; sticky: only destroy is valid after */
#define POND_EBUSY    (-4)  /* server: the stream can never fit the budget, or the    */
                            /* stream cap is reached                                 */
#define POND_ECANCELED (-5) /* server: a queued block of a stream closed before it    */
                            /* was admitted; the block never ran                     */

/* Precision forms. */
#define POND_FP32   0  /* float32 storage and arithmetic                                   */
#define POND_MIXED  1  /* float16 storage and twiddles as POND_HALF, with every radix-16
                          butterfly of the transforms of 64 points and more (columns) and
                          1024 points and more (rows) computed as a 16-point DFT matrix
                          product on the matrix cores (float16 operands, float32
                          accumulation, rounded once to float16); the same power-of-two
                          stage scaling and measured power gain as POND_HALF; chirp and
                          fold phases float64                                              */
#define POND_MIXED_VALU 2  /* float16 storage between passes, every butterfly in float32
                              vector arithmetic                                            */
#define POND_HALF   3  /* float16 storage and packed float16 vector arithmetic (two halves per
                          instruction) for every butterfly, twiddle and the chirp multiply;
                          forward transforms normalised stage by stage; detection and fold
                          in float32 from the float16 pair; chirp and fold phases float64  */
#define POND_BF16   4  /* bfloat16 storage between passes (8-bit significand), every
                          butterfly in float32 vector arithmetic: a reported variant of
                          POND_MIXED_VALU for single-DM plans of complex input, not held to
                          the float16 forms' accuracy                                      */

/* Status bits reported by pond_plan_query().status (sticky until flush). */
#define POND_STATUS_NONFINITE  1u  /* a detected power was inf or NaN (fp16 overflow)        */
#define POND_STATUS_RANGE      2u  /* a power exceeded the fixed-point fold accumulator range */

/* Plan geometry and stream position, filled by pond_plan_query. */
typedef struct pond_info {
    int64_t nfft;          /* FFT length                                          */
    int64_t n_front;       /* ceil(delta_hi * fs): samples dropped at block front  */
    int64_t discard;       /* samples dropped per block (front + back)             */
    int64_t hop;           /* outputs per block = nfft - discard                   */
    int64_t n1, n2;        /* four-step factorisation nfft = n1 * n2 (row x col)   */
    int64_t samples_in;    /* input samples appended since the stream started     */
    int64_t outputs_done;  /* outputs produced since the stream started           */
    int64_t max_batch;     /* blocks per launch                                    */
    double  fs_hz;         /* complex sample rate                                  */
    double  delta_lo_s;    /* delay of band bottom relative to f0                  */
    double  delta_hi_s;    /* advance of band top relative to f0                   */
    double  inv_pfs;       /* 1 / (period_s * fs_hz)                               */
    int32_t nbins;
    int32_t precision;     /* POND_FP32, POND_MIXED, POND_MIXED_VALU, POND_HALF or POND_BF16 */
    uint32_t status;       /* POND_STATUS_* bits (read synchronously)              */
    int32_t input_kind;    /* POND_INPUT_*                                         */
    double  power_gain;    /* POND_HALF: measured power gain of the plan's float16 */
                           /* arithmetic, divided out of every detected power     */
                           /* (1.0 in the other forms)                            */
} pond_info;

/*
 * The overlap-save geometry pond_plan_create would use, without creating a
 * plan (host arithmetic only): n_front, discard and hop of a block of nfft
 * samples (rule above; any output pointer may be NULL).  POND_EINVAL for
 * invalid arguments or when hop would not be positive.
 */
int32_t pond_geometry(double f0_mhz, double bw_mhz, double dm, int64_t nfft,
                      int64_t* n_front, int64_t* discard, int64_t* hop);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the whole
 * path of pond_plan_create_ex + pond_dedisperse_series + the end-of-stream
 * call, with subint_nsamp = 0, over ONE resident segment, allocating
 * nothing.  Every buffer the kernels need beyond the arguments (stage
 * twiddles, the middle-pass table, block work area, fold partials,
 * accumulators, status) lives in a static device array of
 * POND_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until
 * the process ends.  All calls on one GPU share that array: calls that
 * overlap on one GPU race (serialise them, e.g. on one stream).
 *   iq        device, 2*nsamp int8 (I, Q), the whole segment
 *   precision POND_FP32 or POND_MIXED_VALU (the float16-arithmetic forms
 *             need a per-plan gain measurement, which allocates)
 *   nfft      power of two in [2^10, 2^POND_NOALLOC_MAX_LOG2N]
 *   nbins     [1, POND_NOALLOC_MAX_BINS]
 *   decim     as pond_dedisperse_series
 *   profile   device, nbins float32: mean power per bin of every output
 *   series    device, series_cap floats (NULL only if no group completes)
 * Outputs cover every fully covered overlap-save block (Sec. 3.7), as the
 * plan would.  Returns the number of series values written (outputs /
 * decim), or POND_EINVAL (arguments, sizes beyond the limits) /
 * POND_EDEVICE.  Asynchronous on hip_stream; no host synchronisation.
 */
#define POND_NOALLOC_SCRATCH_BYTES (64ll << 20)
#define POND_NOALLOC_MAX_LOG2N 20
#define POND_NOALLOC_MAX_BINS 8192
int64_t pond_dedisperse_segment_noalloc(double f0_mhz, double bw_mhz, double dm, int64_t nfft,
                                        int32_t nbins, double period_s, int32_t precision,
                                        const int8_t* iq, int64_t nsamp, int32_t decim,
                                        float* profile, float* series, int64_t series_cap,
                                        void* hip_stream);

/* Input kinds of a plan (pond_info.input_kind).  For a real-input plan the
   counts of pond_info are in real samples (nfft, n_front, discard, hop,
   samples_in, outputs_done), fs_hz is the real sample rate 2 bw, and
   n1 * n2 = nfft / 2 factors the packed transform. */
#define POND_INPUT_COMPLEX   0
#define POND_INPUT_REAL_LSB  1
#define POND_INPUT_REAL_USB  2

/*
 * Create a plan (plain FP32 form).
 *   f0_mhz   band centre, sky MHz (> bw_mhz/2)
 *   bw_mhz   complex bandwidth = sample rate in Msps (> 0)
 *   dm       dispersion measure, pc cm^-3, finite, >= 0
 *   nfft     FFT length, power of two in [2^10, 2^27]; rows of the four-step
 *            factorisation (n1 = nfft / 2^10) longer than 2^14, i.e. nfft of
 *            2^25 and more, are themselves transformed in four steps (a
 *            column pass of length n1 / 2^13 and sub-rows of 2^13), which
 *            adds one read and one write of the block per pass
 *   nbins    profile bins in [1, 65536]
 *   period_s folding period in seconds, finite, period_s * fs >= 1
 * Geometry: n_front = ceil(delta_hi fs), s = n_front + ceil(delta_lo fs),
 * discard = next_pow2(max(s,16)) if that is <= nfft/2, else s rounded up to
 * a multiple of 16 (0 when s = 0); hop = nfft - discard must be > 0
 * (Sec. 3.7: the filter must be longer than the smear, cyclic edges dropped).
 * Returns NULL on invalid arguments, allocation failure or device failure;
 * pond_create_status() then tells which.
 */
pond_plan* pond_plan_create(double f0_mhz, double bw_mhz, double dm,
                            int64_t nfft, int32_t nbins, double period_s);

/*
 * As pond_plan_create with a precision form (POND_FP32, POND_MIXED,
 * POND_MIXED_VALU, POND_HALF or POND_BF16) and a cap on overlap-save blocks
 * per launch:
 * max_batch > 0 is used as given; POND_BATCH_AUTOTUNE has the plan time its
 * own launch sequence (K1, middle pass, K3 with the series, fold) on
 * pseudo-random int8 input streamed from a ring of 1 GiB (temporarily
 * allocated, less if the device lacks six times that free; each timed
 * run reads samples that no earlier run left in the caches) at 1, 2, 3,
 * 4, 6, 8, 12, 16, 24 and 32 blocks per launch (those
 * whose work area fits in min(4 GiB, a third of the free device memory),
 * plus the default) during creation and
 * keep the fastest per block, a larger launch winning only by more than 0.5%;
 * other values <= 0 pick the default (2^29 bytes of work area, 1 .. 16
 * blocks).  With the environment variable POND_AUTOTUNE_CACHE naming a
 * text file, a choice already measured for the same device, nfft, form,
 * input kind and histogram placement is read from it instead, and new
 * choices are appended (one line each; the last matching line wins).
 */
#define POND_BATCH_AUTOTUNE (-1)
pond_plan* pond_plan_create_ex(double f0_mhz, double bw_mhz, double dm,
                               int64_t nfft, int32_t nbins, double period_s,
                               int32_t precision, int32_t max_batch);

/*
 * The autotuner's result for a plan created with POND_BATCH_AUTOTUNE: the
 * blocks per launch it chose and their measured time per block (ms), the
 * default rule's batch and its measured time per block, and whether the
 * choice came from the cache (1; its times are those of the measuring run).
 * POND_EINVAL for a null plan or one created without the tuner.
 */
int32_t pond_plan_autotune(const pond_plan* p, int32_t* batch, double* ms_per_block,
                           int32_t* default_batch, double* default_ms_per_block,
                           int32_t* from_cache);

/* Status of the last pond_plan_create / _ex call on this thread. */
int32_t pond_create_status(void);

/*
 * Append nsamp samples (iq: device, 2*nsamp int8, I then Q) and fold every
 * newly completed output.  subint_nsamp is S above; it must stay the same
 * for the whole stream (the first call fixes it).  Every sub-integration
 * that completes during the call is written, in order, as nbins float32
 * mean powers at profiles[j*nbins ...] (device, capacity max_profiles
 * profiles).
 * iq == NULL with nsamp == 0 ends the stream: the open sub-integration, if
 * it holds any output, is written as one profile, and the plan returns to
 * an empty stream (position 0) keeping its geometry.
 * Returns the number of profiles written, or POND_EINVAL (null plan,
 * nsamp < 0, iq NULL or misaligned with nsamp > 0, S changed mid-stream,
 * too little profile capacity -- all checked before any work),
 * POND_ENOMEM, or POND_EDEVICE.
 */
int64_t pond_dedisperse_fold(pond_plan* p, const int8_t* iq, int64_t nsamp,
                             int64_t subint_nsamp, float* profiles,
                             int64_t max_profiles, void* hip_stream);

/*
 * pond_dedisperse_fold plus, in the same pass, the detected series summed
 * over decim consecutive outputs (decim in {1, 2, 4, 8, 16}; decim <= 0
 * means round(bw_mhz) outputs, i.e. 1 us (Sec. 4), which must then be one
 * of those values, else POND_EINVAL).  Group i covers outputs
 * [decim*i, decim*i + decim); every group completed by this call is
 * written in order to series (device, capacity series_cap floats) and the
 * count to *n_series_out (host; may be NULL).  series may be NULL only if
 * series_cap is 0 and no group completes.
 */
int64_t pond_dedisperse_series(pond_plan* p, const int8_t* iq, int64_t nsamp,
                               int64_t subint_nsamp, float* profiles,
                               int64_t max_profiles, int32_t decim,
                               float* series, int64_t series_cap,
                               int64_t* n_series_out, void* hip_stream);

/*
 * Frequency-domain taper of the inverse filter (Sec. 3.7: the inverse ISM
 * response is applied together with a taper against leakage of the square
 * window; the paper does not give the taper).  alpha in [0, 1] is the edge
 * fraction of a Tukey window over baseband frequency f in [-bw/2, bw/2]:
 * w(f) = 1 for |f| <= (1 - alpha) bw/2, else
 * (1 + cos(pi (|f| - (1 - alpha) bw/2) / (alpha bw/2))) / 2, reaching 0 at
 * the band edge; alpha = 0 (the default of a new plan) is the unit taper.
 * Allowed only at stream position 0 (new or flushed plan); rebuilds the
 * plan's middle-pass table and synchronises the device.  Returns POND_OK,
 * POND_EINVAL (alpha outside [0, 1], or samples already appended) or
 * POND_EDEVICE.
 */
int32_t pond_plan_set_taper(pond_plan* p, double alpha);

/*
 * Geometry and stream position.  Synchronises the plan's last stream to
 * read the device status word.  Returns POND_OK or an error code.
 */
int32_t pond_plan_query(pond_plan* p, pond_info* out);

/*
 * What a pond_dedisperse_fold / _series call appending nsamp samples would
 * produce from the plan's current position: the number of profiles it
 * writes and the number of new outputs (series groups = n_outputs / decim).
 * nsamp == 0 reports the flush (n_profiles 0 or 1, n_outputs 0).  Host
 * arithmetic only.  Returns POND_OK or POND_EINVAL.
 */
int32_t pond_plan_expect(const pond_plan* p, int64_t nsamp, int64_t subint_nsamp,
                         int64_t* n_profiles, int64_t* n_outputs);

/*
 * Per-kernel device time, for measurement.  Kernels, in launch order:
 *   0  int8 unpack + forward column FFTs
 *   1  twiddle + forward row FFT + chirp + inverse row FFT + twiddle
 *   2  inverse column FFTs + detection + decimation + fold partials
 *   3  fold partial reduction (the partials of up to four K3 launches are
 *      queued and reduced by one launch; `blocks` counts the blocks whose
 *      partials each reduction launch took)
 *   4  profile finalisation
 * With timing on, every launch of the plan is bracketed by two hipEvents
 * on the call's stream; pond_plan_kernel_times synchronises and returns the
 * sums since timing was (re)enabled.
 */
#define POND_NKERNELS 5
typedef struct pond_kernel_times {
    double  ms[POND_NKERNELS];        /* summed event time per kernel        */
    int64_t launches[POND_NKERNELS];  /* launches per kernel                 */
    int64_t blocks[POND_NKERNELS];    /* overlap-save blocks those launches processed */
} pond_kernel_times;

/* Enable (1) or disable (0) per-kernel timing; clears the sums. */
int32_t pond_plan_set_timing(pond_plan* p, int32_t enable);

/* Sums since timing was enabled (synchronises the plan's stream). */
int32_t pond_plan_kernel_times(pond_plan* p, pond_kernel_times* out);

/* Destroy a plan (NULL-safe); waits for the plan's pending work. */
void pond_plan_destroy(pond_plan* p);

/*
 * Real two-channel input (the paper's own receiver path, Sec. 3.1 and
 * Sec. 3.2: two real-sampled channels A and B of one polarisation, added
 * in phase, x[r] = A[r] + B[r], at the real sample rate 2 bw).
 *   raw: device, int8 interleaved A0 B0 A1 B1 ..., 2 bytes per real
 *        sample, 4-byte aligned.
 * Block b covers real samples [b*hop, b*hop + nfft) (nfft, hop, n_front in
 * real samples: twice the complex plan's at the same f0, bw, dm and
 * nfft/2).  Its real spectrum bins k = 0..nfft/2 (baseband k bw/(nfft/2),
 * from 0 to bw) are multiplied by the inverse ISM response of Eq. (4) at
 * sky frequency f0 + f:
 *   POND_USB  f = k bw/(nfft/2) - bw/2,  factor exp(-2 pi i turns(f))
 *   POND_LSB  f = bw/2 - k bw/(nfft/2),  factor exp(+2 pi i turns(f))
 *             (the lower sideband runs backwards, so the phase is conjugated)
 * with turns(f) = dm f^2 / (2.41e-10 f0^2 (f0 + f)) in float64 reduced mod
 * 1 turn, times the taper; the factors of bins 0 and nfft/2 keep only their
 * real part.  The inverse real transform (1/nfft) gives the dedispersed
 * real voltage y; the detected output of real sample r is y[r]^2 (r =
 * b*hop + j, j in [0, hop), input sample r + n_front).  Series groups sum
 * decim consecutive outputs; the fold takes x = (r + n_front) / (P 2 bw)
 * and sub-integrations of S real samples, as above.
 * Computed as a packed complex transform of length nfft/2 (element m =
 * x[2m] + i x[2m+1]): forward, split into the real transform's bins,
 * filter, recombine, inverse.
 */
#define POND_LSB 0
#define POND_USB 1

/* nfft: real block length, a power of two in [2^11, 2^25]; precision
   POND_FP32 or POND_MIXED_VALU; sideband POND_LSB or POND_USB; the rest as
   pond_plan_create_ex.  NULL on failure (pond_create_status()). */
pond_plan* pond_real_plan_create(double f0_mhz, double bw_mhz, double dm, int64_t nfft,
                                 int32_t nbins, double period_s, int32_t precision,
                                 int32_t max_batch, int32_t sideband);

/*
 * Append nsamp real samples (raw: device, 2*nsamp int8 A/B pairs; nsamp
 * even) and fold every newly completed output, as pond_dedisperse_series:
 * subint_nsamp (even, fixed for the stream) and decim (2, 4, 8, 16 or 32;
 * <= 0 means round(2 bw_mhz), 1 us of real samples, which must then be one
 * of those values) in real samples; series NULL: fold only.
 * raw == NULL with nsamp == 0 ends the stream.  Returns the number of
 * profiles written or an error code; only for real-input plans (the
 * complex entry points refuse them, and this one refuses complex plans).
 */
int64_t pond_real_dedisperse(pond_plan* p, const int8_t* raw, int64_t nsamp,
                             int64_t subint_nsamp, float* profiles, int64_t max_profiles,
                             int32_t decim, float* series, int64_t series_cap,
                             int64_t* n_series_out, void* hip_stream);

/* pond_plan_expect for a real-input plan, in real samples (nsamp and
   subint_nsamp even). */
int32_t pond_real_expect(const pond_plan* p, int64_t nsamp, int64_t subint_nsamp,
                         int64_t* n_profiles, int64_t* n_outputs);

/*
 * DM-trial search (one stream dedispersed and folded at many trial DMs).
 * Each trial t is processed exactly as a single-DM plan of FFT length
 * N_t = clamp(2 discard_t, nfft_min, nfft_max) (discard_t by the plan
 * rule above), except that all trials of one N_t share one block grid with
 * hop = N_t / 2 and therefore one forward transform per block; each keeps
 * its own n_front_t.  dms (host, ntrials values >= 0), nfft_min/nfft_max
 * powers of two in [2^10, 2^24]; every trial needs discard_t <= nfft_max/2.
 * precision as for pond_plan_create_ex.  Device memory per length group:
 * the blocks of one launch twice (spectrum, one trial's output), the
 * four-step twiddles and one float64 table of the chirp's turns per unit DM
 * of each bin, shared by the group's trials (a trial's chirp is
 * exp(-2 pi i frac(DM g_k)), formed as the inverse rows read the spectrum;
 * its sine and cosine in float32 after the float64 reduction).  Returns
 * NULL on invalid arguments or allocation/device failure.
 */
typedef struct pond_search pond_search;
pond_search* pond_search_create(double f0_mhz, double bw_mhz, const double* dms, int32_t ntrials,
                                int32_t nbins, double period_s, int64_t nfft_min, int64_t nfft_max,
                                int32_t precision);

/*
 * As pond_search_create with blocks per launch for every length group:
 * max_batch > 0 as given; POND_BATCH_AUTOTUNE tunes each group as
 * pond_plan_create_ex does (its forward pass and two trials' inverse
 * passes timed on pseudo-random input; POND_AUTOTUNE_CACHE as there);
 * other values <= 0 the default (2^28 bytes of spectrum, 1 .. 16 blocks).
 */
pond_search* pond_search_create_ex(double f0_mhz, double bw_mhz, const double* dms, int32_t ntrials,
                                   int32_t nbins, double period_s, int64_t nfft_min, int64_t nfft_max,
                                   int32_t precision, int32_t max_batch);

/* The autotuner's result for the length group of FFT length nfft (see
   pond_plan_autotune); POND_EINVAL if there is no such group or it was not
   tuned. */
int32_t pond_search_autotune(const pond_search* s, int64_t nfft, int32_t* batch, double* ms_per_block,
                             int32_t* default_batch, double* default_ms_per_block,
                             int32_t* from_cache);

/*
 * Fold one whole stream (iq: device, 2*nsamp int8) at every trial DM and
 * write profiles (device, ntrials*nbins float32): trial t's mean detected
 * power per bin over all outputs of its fully covered blocks (one open-ended
 * sub-integration; fold phase as above with that trial's n_front).
 * Asynchronous on hip_stream.  Returns POND_OK, POND_EINVAL or POND_EDEVICE.
 */
int32_t pond_search_run(pond_search* s, const int8_t* iq, int64_t nsamp, float* profiles,
                        void* hip_stream);

/* FFT length, n_front and hop of trial t. */
int32_t pond_search_trial(const pond_search* s, int32_t t, int64_t* nfft, int64_t* n_front,
                          int64_t* hop);

/* Destroy a search (NULL-safe); waits for its pending work. */
void pond_search_destroy(pond_search* s);

/*
 * Real-time serving of many streams on one device (continuous batching).
 *
 * A server admits streams, each a plan of its own with the usual geometry,
 * against a device-memory budget.  An admitted stream keeps its overlap
 * tail and fold accumulators on the device between blocks.  Blocks of int8
 * samples arrive in HOST memory and are submitted as they arrive.  A block
 * is dispatched at once if its stream has fewer than two blocks on the
 * device: copy to the device, dedispersion + fold (Sec. 3.7), copy of the
 * completed profiles back, on the stream's own non-blocking HIP stream.
 * Otherwise it waits in the stream's queue until poll() finds a slot free.
 * Blocks of different streams thus overlap on the device, and each stream's
 * blocks run in order, so its results are those of the same blocks passed
 * to pond_dedisperse_fold one after another on a plan of its own.
 *
 * The server is single-threaded: call it from one host thread.  Host block
 * memory must stay valid and unmodified until poll() has reported that
 * block; pinned memory (hipHostMalloc) makes the copy asynchronous,
 * pageable memory makes the submitting call wait for the copy.
 */
typedef struct pond_server pond_server;

typedef struct pond_stream_desc {
    double  f0_mhz, bw_mhz, dm, period_s;  /* as pond_plan_create                  */
    int64_t nfft;                          /* as pond_plan_create                  */
    int64_t subint_nsamp;                  /* S of the stream (0 = one open-ended)  */
    int64_t max_block_nsamp;               /* largest block the stream will submit */
    int32_t nbins;
    int32_t precision;                     /* POND_FP32 / POND_MIXED / POND_MIXED_VALU / POND_HALF */
} pond_stream_desc;

typedef struct pond_completion {
    int64_t ticket;       /* as returned by pond_server_submit                        */
    int32_t stream;       /* stream id                                                */
    int32_t status;       /* POND_OK or the error that ended the stream               */
    int64_t n_profiles;   /* sub-integrations the block completed                     */
    double  latency_us;   /* host clock: submission to completion seen by the server  */
    double  device_us;    /* device time from the block's copy-in to its copy-out     */
} pond_completion;

/* A server on the current device with a budget in bytes of device memory
   and a cap on open streams.  NULL on bad arguments. */
pond_server* pond_server_create(int64_t hbm_budget_bytes, int32_t max_streams);

/* Device bytes a stream with this description holds while open (default
   blocks per launch), or POND_EINVAL. */
int64_t pond_server_stream_bytes(const pond_stream_desc* d);

/* Open a stream: returns its id (>= 0).  The stream is admitted at once if
   it fits the budget left (with fewer blocks per launch tried first);
   otherwise it waits, first come first, and is admitted by a later open,
   poll or close once enough memory has been returned (its admission is
   then reported by poll() as a completion with ticket POND_TICKET_ADMITTED).
   Blocks may be submitted to a waiting stream; they run after admission.
   POND_EBUSY if the stream would not fit even an empty server or the cap on
   open plus waiting streams is reached, POND_EINVAL for an invalid
   description, POND_ENOMEM / POND_EDEVICE if its admission failed. */
int32_t pond_server_open(pond_server* s, const pond_stream_desc* d);

#define POND_TICKET_ADMITTED (-1)  /* pond_completion.ticket of an admission       */
#define POND_STREAM_WAITING 0      /* opened, waiting for budget                   */
#define POND_STREAM_OPEN    1      /* admitted: plan and slots on the device       */
#define POND_STREAM_CLOSED  2      /* closed (or its admission failed)             */

/* State of a stream id (POND_STREAM_*), or POND_EINVAL. */
int32_t pond_server_stream_state(const pond_server* s, int32_t stream);

/* Submit the stream's next block (host_iq: 2*nsamp int8, 0 < nsamp <=
   max_block_nsamp) to an open or waiting stream.  Returns a ticket (>= 0)
   or an error. */
int64_t pond_server_submit(pond_server* s, int32_t stream, const int8_t* host_iq, int64_t nsamp);

/* Report completed blocks (up to max_out, in completion order per stream)
   and dispatch queued blocks into freed slots.  With wait != 0, waits until
   at least one block completes or nothing is on the device.  Returns the
   number of completions written, or POND_EINVAL. */
int32_t pond_server_poll(pond_server* s, pond_completion* out, int32_t max_out, int32_t wait);

/* Move up to max_profiles of the stream's completed profiles (oldest
   first, nbins float32 each) to host_out and drop them from the server;
   valid before and after close.  Returns the number moved. */
int64_t pond_server_take_profiles(pond_server* s, int32_t stream, float* host_out, int64_t max_profiles);

/* End a stream: run its queued blocks, append the open sub-integration as
   its last profile, free its device memory and return it to the budget
   (which may admit waiting streams).  A stream still waiting for admission
   is dropped: its queued blocks complete with POND_ECANCELED.  Completions
   seen meanwhile are reported by the next poll().  Returns POND_OK or the
   error that ended the stream. */
int32_t pond_server_close(pond_server* s, int32_t stream);

/* Budget in use, budget, open streams and blocks queued or on the device. */
int32_t pond_server_query(const pond_server* s, int64_t* used_bytes, int64_t* budget_bytes,
                          int32_t* open_streams, int64_t* queued_blocks);

/* Destroy a server (NULL-safe): waits for and frees every open stream. */
void pond_server_destroy(pond_server* s);

/*
 * Incoherent dedispersion with an FFT filterbank (the AID pulsar mode,
 * Sec. 3.4 / Sec. 3.4.1; Eq. (2) gives its residual smear, Eq. (3) its
 * per-channel delays).  Input as above (complex int8 I/Q, device).  The
 * stream is cut into back-to-back blocks of nchan samples; each block's
 * nchan-point spectrum is squared, nint consecutive spectra are summed
 * (integrated sample t_s = nchan nint / fs); channel c (baseband frequency
 * fftfreq(nchan) * bw, sky f0 + f) is delayed by
 * d_c = floor((1/2.41e-4) DM (f^-2 - f0^-2) / t_s + 1/2) integrated
 * samples, referred to f0; dedispersed output m (m >= 0) is the sum over
 * channels of channel c's sample m + d_c - d_min, and exists where every
 * channel covers it.  Output m has time (m - d_min) t_s and is folded with
 * x = (m - d_min) nchan nint / (P fs) as the coherent mode's outputs.
 */
typedef struct pond_aid pond_aid;

/* nchan: power of two in [64, 4096]; nint in [1, 65536]; other arguments as
   pond_plan_create.  NULL on invalid arguments or device failure. */
pond_aid* pond_aid_create(double f0_mhz, double bw_mhz, double dm, int32_t nchan,
                          int32_t nint, int32_t nbins, double period_s);

/* For a segment of nsamp samples: integrated spectra, dedispersed outputs,
   the smallest and largest channel delays and t_s (any pointer may be
   NULL).  Host arithmetic only. */
int32_t pond_aid_geometry(const pond_aid* a, int64_t nsamp, int64_t* n_spectra,
                          int64_t* n_series, int32_t* d_min, int32_t* d_max, double* t_s);

/* Process one resident segment (nothing is carried between calls): the
   folded profile (nbins float32 means, device) and, if series is not NULL,
   the dedispersed series (device, capacity series_cap >= n_series).
   Returns n_series or POND_EINVAL / POND_ENOMEM / POND_EDEVICE.
   Asynchronous on hip_stream. */
int64_t pond_aid_run(pond_aid* a, const int8_t* iq, int64_t nsamp, float* profile,
                     float* series, int64_t series_cap, void* hip_stream);

/* Destroy (NULL-safe); waits for the last call's work. */
void pond_aid_destroy(pond_aid* a);

/*
 * Device-to-device copy of `bytes` (a multiple of 16; dst and src device
 * pointers, 16-byte aligned, not overlapping) with the library's own
 * streaming kernel, asynchronous on hip_stream.  For measurement: the
 * bandwidth it reaches is the achievable HBM rate that the kernels' byte
 * counts are set against, beside the device's nominal peak.  Returns POND_OK,
 * POND_EINVAL or POND_EDEVICE.
 */
int32_t pond_copy_device(void* dst, const void* src, int64_t bytes, void* hip_stream);

/* Static text for a return code. */
const char* pond_strerror(int64_t code);

#ifdef __cplusplus
}
#endif

#endif /* POND_H */
