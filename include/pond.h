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
 *     interleaved, in DEVICE memory, 2-byte aligned.
 *   - Block b of the stream covers input samples [b*hop, b*hop + nfft).
 *     Its kept outputs are outputs m = b*hop + j, j in [0, hop); output m
 *     is input sample m + n_front, referred to arrival at f0.  Only fully
 *     covered blocks produce outputs.
 *   - Each spectrum bin k (frequency f_k = k*bw/nfft, k >= nfft/2 taken as
 *     k - nfft) is multiplied by exp(-2 pi i turns_k) with
 *     turns_k = dm f_k^2 / (2.41e-10 f0^2 (f0 + f_k)), the inverse of the
 *     ISM response of Eq. (4) with the dispersion constant of Eq. (1).
 *     The phase is evaluated and reduced mod 1 turn in float64.
 *   - Forward transform unnormalised, inverse with 1/nfft; no taper.
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

/* Precision forms. */
#define POND_FP32   0  /* float32 storage and arithmetic                                   */
#define POND_MIXED  1  /* float16 storage between passes; the radix-16 stages of the column
                          passes run as 16-point DFT matrix products on the matrix cores
                          (float16 operands, float32 accumulation, power-of-two stage
                          scaling); chirp and fold phases stay float64                      */
#define POND_MIXED_VALU 2  /* float16 storage between passes, every butterfly in float32
                              vector arithmetic                                            */

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
    int32_t precision;     /* POND_FP32, POND_MIXED or POND_MIXED_VALU             */
    uint32_t status;       /* POND_STATUS_* bits (read synchronously)              */
    int32_t reserved;
} pond_info;

/*
 * Create a plan (plain FP32 form).
 *   f0_mhz   band centre, sky MHz (> bw_mhz/2)
 *   bw_mhz   complex bandwidth = sample rate in Msps (> 0)
 *   dm       dispersion measure, pc cm^-3, finite, >= 0
 *   nfft     FFT length, power of two in [2^10, 2^24]
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
 * As pond_plan_create with a precision form (POND_FP32, POND_MIXED or
 * POND_MIXED_VALU) and a cap on overlap-save blocks per launch (max_batch
 * <= 0 picks a default).
 */
pond_plan* pond_plan_create_ex(double f0_mhz, double bw_mhz, double dm,
                               int64_t nfft, int32_t nbins, double period_s,
                               int32_t precision, int32_t max_batch);

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
 * means 16, i.e. 1 us at 16 Msps).  Group i covers outputs
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
 *   3  fold partial reduction
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
 * DM-trial search (one stream dedispersed and folded at many trial DMs).
 * Each trial t is processed exactly as a single-DM plan of FFT length
 * N_t = clamp(2 discard_t, nfft_min, nfft_max) (discard_t by the plan
 * rule above), except that all trials of one N_t share one block grid with
 * hop = N_t / 2 and therefore one forward transform per block; each keeps
 * its own n_front_t.  dms (host, ntrials values >= 0), nfft_min/nfft_max
 * powers of two in [2^10, 2^24]; every trial needs discard_t <= nfft_max/2.
 * precision as for pond_plan_create_ex.  Returns NULL on invalid arguments
 * or allocation/device failure.
 */
typedef struct pond_search pond_search;
pond_search* pond_search_create(double f0_mhz, double bw_mhz, const double* dms, int32_t ntrials,
                                int32_t nbins, double period_s, int64_t nfft_min, int64_t nfft_max,
                                int32_t precision);

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

/* Static text for a return code. */
const char* pond_strerror(int64_t code);

#ifdef __cplusplus
}
#endif

#endif /* POND_H */
