/*
 * cobalt.h - C ABI of the MI355X FX correlator (the correlator hot path of LOFAR's Cobalt,
 * arXiv 1801.04834).
 *
 * One plan per observation setting.  Per ~1 s block of station samples the library runs
 *   F stage: unpack -> polyphase FIR (history carried) -> C-point FFT -> fine delay
 *            compensation + bandpass correction -> transpose to the cross-station layout
 *            (+ precision conversion),
 *   X stage: V[a][b] = sum_t Z_a(t) conj(Z_b(t)) over all station pairs and polarisations,
 * as described in the paper's "Signal processing with GPU kernels" (sec. 7.5) and
 * "Processing steps" (sec. 3.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named d_* are DEVICE pointers (HIP global memory on the plan's device) owned
 *    by the caller; they must be 16-byte aligned.  Pointers named h_* are host pointers;
 *    the library copies what it needs before returning, so the caller may reuse them at
 *    once.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Every call
 *    enqueues work and returns; results are ready when the stream reaches that point.
 *  - Stateful calls (cobalt_correlate(_ex), cobalt_channelize(_ex), cobalt_beamform,
 *    cobalt_reset_history: they use the
 *    FIR history, the delay staging and, for cobalt_correlate, the plan's channelised
 *    buffer) are ordered among themselves even across streams (the plan waits on its
 *    previous stateful call's completion event); two host threads must not make stateful
 *    calls on one plan at the same time (COBALT_EBUSY).
 *  - Stateless calls (cobalt_correlate_channelized, cobalt_beamform_channelized,
 *    cobalt_apply_gains, cobalt_apply_gains_adjoint) read only the plan's fixed sizes: they are ordered by the
 *    caller's stream alone, may be made from any host thread, and may overlap stateful
 *    calls on other streams (e.g. the X stage of block k with the F stage of block k+1 into
 *    a second channelised buffer).  The caller orders buffer reuse with its own events.
 *  - Different plans may run concurrently.
 *  - Return value: COBALT_OK (0) or a negative COBALT_E* code; cobalt_last_error() gives a
 *    message (thread-local).  No C++ exception crosses this boundary.
 *
 * Notation: S stations (antenna fields), P = 2 polarisations, M = S*P inputs (input index
 * a = s*P + p), SB subbands, C channels, T taps, N samples per input per subband per
 * block, N_c = N / C channel samples, B = S(S+1)/2 baselines (s1 >= s2, autos included).
 *
 * Layouts (row-major, last index fastest)
 * ---------------------------------------
 *  input block   [S][P][SB][N] complex samples: int8 pairs (COBALT_CI8), int16 pairs
 *                (COBALT_CI16) or float pairs (COBALT_CF32), (re, im) interleaved.
 *  channelised   K-blocked, per channel (sb*C + c): n_kb = pitch/32 blocks of 32 channel
 *                samples, each block holding planes x M rows x 32 samples:
 *                 FP32 mode      [SB][C][n_kb][M][32] float (re, im)
 *                 FP16-split     [SB][C][n_kb][2][M][32] _Float16 (re, im); plane 0 = hi,
 *                                plane 1 = lo, hi + lo = 2^k * Z (k = fp16_prescale_log2)
 *                 INT8 mode      [SB][C][n_kb][M][32] int8 (re, im), values in [-127, 127]
 *                Sample j of input row a sits in block j/32 at position j%32.  pitch = N_c
 *                rounded up to a multiple of 32; positions j >= N_c are written as zero by
 *                the F stage and ignored by the X stage.  One channel's K block is one
 *                contiguous run (the X stage streams it; the F stage writes neighbouring
 *                rows of it from concurrent waves).
 *  visibilities  [SB][C][B][4] complex: float (re, im) in FP32 / FP16-split modes,
 *                int32 (re, im) raw integer sums in INT8 mode.  Baseline index
 *                b(s1, s2) = s1(s1+1)/2 + s2 for s1 >= s2; pol pair q = 2*p1 + p2
 *                (XX, XY, YX, YY); entry = sum_j Z[s1*P+p1][j] * conj(Z[s2*P+p2][j]).
 */
#ifndef COBALT_H
#define COBALT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------------------ */
#define COBALT_OK            0
#define COBALT_EINVAL       -1   /* bad argument: sizes, NULL pointers, N % C != 0 ...   */
#define COBALT_EUNSUPPORTED -2   /* valid but not built: C not 64/256, T != 16, P != 2, M > 160 in MFMA modes */
#define COBALT_EOVERFLOW    -3   /* INT8 mode with N_c * 2 * 127^2 >= 2^31 (int32 sums), or an
                                    FP16-split prescale that full-scale samples would overflow */
#define COBALT_ENOMEM       -4   /* device or pinned host allocation failed              */
#define COBALT_EBUSY        -5   /* another host thread is inside a call on this plan    */
#define COBALT_EDEVICE      -6   /* HIP runtime error; see cobalt_last_error()           */

/* ---- sample types and X-stage modes -------------------------------------------------- */
#define COBALT_CI8   1   /* complex int8 station samples (8-bit mode)                      */
#define COBALT_CI16  2   /* complex int16 station samples (16-bit mode)                    */
#define COBALT_CF32  3   /* complex float32 samples (exact test signals)                   */

#define COBALT_X_FP32        0   /* FP32 channelised data, FP32 VALU correlator (plain form) */
#define COBALT_X_FP16_SPLIT  1   /* FP16 hi/lo planes, FP16 MFMA (hh+hl+lh), FP32 accumulate */
#define COBALT_X_INT8        2   /* int8 requantised data, int8 MFMA, int32 accumulate       */

typedef struct cobalt_plan cobalt_plan;   /* opaque: workspace, FIR history, tables */

/* Observation setting.  Host arrays are copied by cobalt_plan_create. */
typedef struct cobalt_config {
    int32_t n_stations;          /* S >= 1                                                */
    int32_t n_pols;              /* P, must be 2                                          */
    int32_t n_subbands;          /* SB >= 1                                               */
    int32_t n_channels;          /* C: 64 or 256 (the two channel counts built)           */
    int32_t n_taps;              /* T, 16 (the only tap count built)                      */
    int32_t sample_type;         /* COBALT_CI8 | COBALT_CI16 | COBALT_CF32                */
    int32_t x_mode;              /* COBALT_X_FP32 | COBALT_X_FP16_SPLIT | COBALT_X_INT8   */
    int32_t fp16_prescale_log2;  /* k in [-24, 24]: FP16-split stores 2^k * Z; V is scaled
                                    back by 2^-2k (exact).  Ignored in other modes.  For
                                    CI8 / CI16 samples k must not exceed the bound that
                                    cobalt_fp16_prescale_max reports (else EOVERFLOW), so
                                    no valid input overflows FP16; for CF32 samples the
                                    caller keeps 2^k |Z| <= 65504, larger components are
                                    stored saturated at +-65504.                          */
    int64_t samples_per_block;   /* N >= 0, multiple of C (196608 for ~1 s blocks)        */
    double  sample_rate_hz;      /* f_s > 0, subband sample rate (195312.5)               */
    float   requant_gain;        /* g > 0: INT8 mode stores clamp(rint(g * Z), +-127)      */
    int32_t reserved0;           /* must be 0                                             */
    const float*  h_fir;         /* [T*C] prototype FIR; output j, phase p uses
                                    sum_t h[t*C+p] * x[(j-T+1+t)*C + p]                   */
    const float*  h_bandpass;    /* [C] real bandpass correction per channel, or NULL (1) */
    const double* h_subband_freq_hz; /* [SB] sky centre frequency of each subband (Hz)    */
} cobalt_config;

/* Sizes of one plan (filled by cobalt_plan_query). */
typedef struct cobalt_plan_info {
    int64_t n_channel_samples;   /* N_c = N / C                                           */
    int64_t chan_pitch;          /* channel samples per channelised row (>= N_c)          */
    int64_t n_baselines;         /* B = S(S+1)/2                                          */
    int64_t input_bytes;         /* bytes of one input block                              */
    int64_t chan_bytes;          /* bytes of the channelised buffer                       */
    int64_t vis_bytes;           /* bytes of the visibility buffer                        */
    int64_t workspace_bytes;     /* device bytes held by the plan                         */
    int64_t useful_cmacs;        /* complex MACs per block: B * 4 * SB * C * N_c          */
} cobalt_plan_info;

/* Create a plan on the current HIP device: validates cfg, allocates the device workspace
 * (channelised buffer, two FIR-history buffers zeroed, tables, delay staging) and copies
 * the host tables.  On success *out owns everything; on failure *out is NULL and nothing
 * is leaked.  Errors: EINVAL, EUNSUPPORTED, EOVERFLOW, ENOMEM, EDEVICE. */
int cobalt_plan_create(const cobalt_config* cfg, cobalt_plan** out);

/* Device bytes cobalt_plan_create would allocate for cfg (for admission by HBM budget).
 * Performs the same validation as create.  Allocates nothing. */
int cobalt_estimate_bytes(const cobalt_config* cfg, size_t* device_bytes);

/* Largest fp16_prescale_log2 for which no CI8 / CI16 input can overflow FP16 in the
 * FP16-split channelised data (sec. 3.2: the fixed-point samples become floats before the
 * chain).  Every channel sample satisfies |Z| <= max_c |b_c| * sum_m |h[m]| * max|x|, with
 * max|x| = 2^15 sqrt(2) (CI16) or 2^7 sqrt(2) (CI8), by the triangle inequality through
 * FIR, DFT, unit-modulus delay phasor and bandpass; an input matched to the signs of the
 * taps reaches it.  *k_max is the largest k with 2^k * bound * (1 + 2^-10) <= 65504, at
 * most 24 (the margin covers the F stage's FP32 rounding).  With the Blackman-windowed sinc
 * of 16 taps (sum |h| = 1.60) and a bandpass peaking at 1.05 this is -1 for CI16 and 7 for
 * CI8.  cfg is validated as for cobalt_plan_create (its x_mode and prescale are ignored).
 * Allocates nothing.  Errors: EINVAL (NULL, invalid cfg, CF32 samples: no fixed bound),
 * EUNSUPPORTED, EOVERFLOW (no k >= -24 is safe). */
int cobalt_fp16_prescale_max(const cobalt_config* cfg, int32_t* k_max);

/* Fill *info with the plan's sizes.  Errors: EINVAL (NULL). */
int cobalt_plan_query(const cobalt_plan* plan, cobalt_plan_info* info);

/* Full FX chain for one block: F stage into the plan's channelised buffer, then X stage
 * into d_vis.  d_in: input block layout; h_delays: [S][2] float64 residual delays in
 * seconds at block start and block end (fine delay compensation, sec. 7.5: phase
 * exp(+2 pi i f_c tau(j)), tau linear in the channel sample j); d_vis: visibilities.
 * Advances the FIR history.  Errors: EINVAL, EBUSY, EDEVICE. */
int cobalt_correlate(cobalt_plan* plan, const void* d_in, const double* h_delays,
                     void* d_vis, void* stream);

/* F stage only: writes the channelised layout to d_chan (caller-owned, chan_bytes).
 * Advances the FIR history exactly like cobalt_correlate.  Errors as cobalt_correlate. */
int cobalt_channelize(cobalt_plan* plan, const void* d_in, const double* h_delays,
                      void* d_chan, void* stream);

/* ---- coarse delay and lost samples ---------------------------------------------------
 * Optional per-block extras of cobalt_correlate_ex / cobalt_channelize_ex.  The paper
 * compensates the whole-sample part of each station's delay by shifting its sample stream
 * (sec. 7.1) and applies only the residual as the fine delay (sec. 7.5); lost input is
 * recorded as metadata of the data product (sec. 3.2, sec. 7.2).  Here:
 *  - Coarse delay: input rows hold row_samples = N + G samples; station s reads its block
 *    window row[g_s .. g_s + N) (g_s = h_coarse_offset[s], 0 <= g_s <= G, shared by both
 *    polarisations and all subbands).  The FIR history carries the end of the previous
 *    window, so changing g_s between blocks repeats or skips samples at the block edge.
 *    h_delays then holds the residual delays.
 *  - Lost samples: d_flags [S][SB][flag_words] uint32, flag_words = ceil(row_samples / 32):
 *    bit k of word w set = sample 32w + k of the row of station s, subband sb is lost (both
 *    polarisations).  A channel sample j is flagged when any sample of its FIR window (the
 *    T*C samples (j-T+1)*C .. (j+1)*C - 1 of the block window, reaching into the previous
 *    block) is lost; flagged channel samples are written as zero to the channelised data, so
 *    they drop out of every visibility.  The plan carries the flags of the last T-1 rows of C
 *    samples to the next block (cleared by cobalt_reset_history; honoured by the plain calls
 *    too).
 *  - Weights: d_weights [SB][B] int32 receives, per baseline, the number of channel samples
 *    valid for both stations (N_c when nothing is lost).
 * Every field may be zero / NULL: row_samples 0 means N, NULL offsets mean 0, NULL flags
 * mean nothing lost, NULL weights are not written. */
typedef struct cobalt_block_ext {
    int64_t         row_samples;       /* samples per input row, >= N; 0 = N                  */
    const int32_t*  h_coarse_offset;   /* host [S], copied before return; NULL = all 0         */
    const uint32_t* d_flags;           /* device [S][SB][flag_words], 4-byte aligned; NULL     */
    int32_t*        d_weights;         /* device [SB][B], 4-byte aligned; NULL                 */
} cobalt_block_ext;

/* cobalt_correlate with coarse delay, lost-sample flags and weights.  d_in: [S][P][SB]
 * [row_samples] complex samples.  ext == NULL is cobalt_correlate.  Errors: EINVAL (an
 * offset outside 0..row_samples-N, misaligned pointers), EBUSY, EDEVICE. */
int cobalt_correlate_ex(cobalt_plan* plan, const void* d_in, const double* h_delays,
                        const cobalt_block_ext* ext, void* d_vis, void* stream);

/* cobalt_channelize with the same extras (flagged channel samples are zero in d_chan). */
int cobalt_channelize_ex(cobalt_plan* plan, const void* d_in, const double* h_delays,
                         const cobalt_block_ext* ext, void* d_chan, void* stream);

/* ---- beamformer ----------------------------------------------------------------------
 * The paper's second pipeline (sec. 7.5, sec. 5): the same front end (a plan with
 * n_channels = 256 is the paper's setting; 64 also works), then per channel
 *   coherent beams   beam[b][p][t] = sum_s w[b][s] Z[s*P + p][t],
 *                    w[b][s] = exp(+2 pi i f_c dtau[b][s])  (phase in FP64, reduced, FP32
 *                    rotation), dtau = extra arrival delay of beam b's direction at station s,
 *   Stokes           I = |X|^2 + |Y|^2, Q = |X|^2 - |Y|^2, U = 2 Re(X conj Y),
 *                    V = 2 Im(X conj Y)  from the polarisations X (p = 0), Y (p = 1),
 *   incoherent       per-station Stokes summed over stations,
 * with Stokes summed over n_int consecutive channel samples.  Requires an FP16-split plan
 * (the products run on matrix cores with hi/lo operands) and at most 56 stations.
 * Output layouts (float, beams fastest: each output sample is one row over the beams):
 *   d_coherent    [SB][C][N_c / n_int][n_stokes][NB]
 *   d_voltages    [SB][C][N_c][P][NBs] complex (re, im); beams NB .. NBs-1 of a row are
 *                 padding: unspecified on return (zeros where a kernel's beam group covers
 *                 them, so that padded rows are written as whole lines), never read
 *   d_incoherent  [SB][C][N_c / n_int][n_stokes]
 * Any output may be NULL (not computed); at least one must be given. */
typedef struct cobalt_beam_params {
    int32_t       n_beams;      /* NB >= 1                                                  */
    int32_t       n_stokes;     /* 1 (I) or 4 (I, Q, U, V)                                  */
    int32_t       n_int;        /* a power of two <= 32 or a multiple of 32; divides N_c    */
    int32_t       voltage_stride; /* NBs, beams per row of d_voltages: 0 means NB, else >= NB
                                   (at most 65536).  A multiple of 16 puts every 16 beams of
                                   a row on whole 128-byte lines, which the output-resolution
                                   transform reads and writes much faster              */
    const double* d_beam_dtau;  /* device [NB][S] seconds, 8-byte aligned                    */
} cobalt_beam_params;

/* F stage (stateful, like cobalt_correlate: advances the FIR history) into the plan's
 * channelised buffer, then the beamformer.  Errors: EINVAL, EUNSUPPORTED (mode, stations),
 * EBUSY, EDEVICE. */
int cobalt_beamform(cobalt_plan* plan, const void* d_in, const double* h_delays, const cobalt_beam_params* beams,
                    void* d_coherent, void* d_voltages, void* d_incoherent, void* stream);

/* Beamformer only, on a caller-provided channelised buffer (FP16-split layout of this plan).
 * Stateless.  Errors: EINVAL, EUNSUPPORTED, EDEVICE. */
int cobalt_beamform_channelized(cobalt_plan* plan, const void* d_chan, const cobalt_beam_params* beams,
                                void* d_coherent, void* d_voltages, void* d_incoherent, void* stream);

/* ---- output resolution of the beams --------------------------------------------------
 * The paper forms beams at 256 channels per subband and then transforms them to the
 * requested output resolution, often 1 or 16 channels per subband (sec. 7.5), trading time
 * resolution for frequency resolution within the subband (sec. 5).  Per subband, beam and
 * polarisation, the 256 channel values of each channel sample j go back to 256 time samples
 *     u[256 j + n] = (1/256) sum_c B[c][j] exp(+2 pi i n (c - 128) / 256),
 * and every group of c_out consecutive samples gets a forward DFT
 *     O[g][c'] = sum_m u[g c_out + m] exp(-2 pi i m (c' - c_out/2) / c_out)
 * (output channel c' ascending in frequency; c_out = 1 is the time series at the subband
 * sample rate).  Layouts (float, beams fastest), G = N_c * 256 / c_out output samples:
 *   d_voltages      [SB][256][N_c][P][NBs] complex: the beamformer's voltage output (beams
 *                   NB .. NBs-1 of a row are padding, never read)
 *   d_out_voltages  [SB][G][c_out][P][NBs] complex (padding beams unspecified on return)
 *   d_out_stokes    [SB][G / n_int][c_out][n_stokes][NB]: Stokes (as for the beamformer) of
 *                   the transformed voltages summed over n_int consecutive output samples */
typedef struct cobalt_transform_params {
    int32_t n_beams;     /* NB >= 1 (as given to the beamformer)                              */
    int32_t c_out;       /* output channels per subband: 1, 2, 4, 8 or 16                     */
    int32_t n_stokes;    /* 1 (I) or 4 (I, Q, U, V); read only when Stokes are requested      */
    int32_t n_int;       /* a power of two up to 256 / c_out; read only when Stokes are requested */
    int32_t voltage_stride; /* beams per row of d_voltages and d_out_voltages (NBs): 0 means NB,
                               else >= NB; the beamformer's voltage_stride of the same voltages */
} cobalt_transform_params;

/* Transform beamformed voltages of a 256-channel plan to c_out channels; either output may
 * be NULL (not computed), not both.  Stateless (ordered by the stream alone).  Errors: EINVAL,
 * EUNSUPPORTED (plan not at 256 channels, c_out, or one subband's voltages of 4 GiB or more:
 * N_c * NBs must stay below 2^20), EDEVICE. */
int cobalt_beam_transform(cobalt_plan* plan, const void* d_voltages, const cobalt_transform_params* params,
                          void* d_out_voltages, void* d_out_stokes, void* stream);

/* X stage only, on a caller-provided channelised buffer in this plan's mode and layout
 * (positions >= N_c are ignored).  Stateless (see above).  Errors: EINVAL, EDEVICE. */
int cobalt_correlate_channelized(cobalt_plan* plan, const void* d_chan, void* d_vis,
                                 void* stream);

/* Zero the FIR history (start of a new observation / after a gap in the stream).
 * Errors: EINVAL, EBUSY, EDEVICE. */
int cobalt_reset_history(cobalt_plan* plan, void* stream);

/* Gain-applied visibilities (FP32 and FP16-split modes): complex gains per input, subband
 * and channel, constant over the block, applied to the channelised samples before the X stage
 * scale each stored entry:  d_vis[sb][c][bl][q] = g[a] conj(g[b]) d_vis0[sb][c][bl][q] with
 * a = 2 s1 + p1, b = 2 s2 + p2.  d_gains: float (re, im) [SB][C][M]; d_vis0, d_vis: the
 * visibility layout (d_vis may equal d_vis0).  Stateless.  Errors: EINVAL, EUNSUPPORTED
 * (INT8 mode), EDEVICE.  (The differentiable correlator of the 16-bit path.) */
int cobalt_apply_gains(cobalt_plan* plan, const void* d_vis0, const void* d_gains, void* d_vis,
                       void* stream);

/* Adjoint of cobalt_apply_gains.  Given the upstream gradient d_grad_vis = dL/dRe V + i dL/dIm V
 * of a real loss L (visibility layout), writes d_grad_gains[sb][c][k] = dL/dRe g_k + i dL/dIm g_k:
 *   sum over stored entries with b = k of conj(G) g[a] V0  +  with a = k of G g[b] conj(V0).
 * Deterministic (fixed summation order, no atomics).  d_grad_gains must not alias the inputs.
 * Errors as cobalt_apply_gains. */
int cobalt_apply_gains_adjoint(cobalt_plan* plan, const void* d_vis0, const void* d_gains,
                               const void* d_grad_vis, void* d_grad_gains, void* stream);

/* Plain device-to-device copy of `bytes` (a multiple of 16; 16-byte aligned pointers) on the
 * current device, 16 bytes per lane.  Reference kernel for calibrating HBM traffic counters
 * and for an HBM readiness check before timing (the paper verifies performance with
 * operational readiness scripts, sec. 8).  Errors: EINVAL, EDEVICE. */
int cobalt_device_copy(void* d_dst, const void* d_src, size_t bytes, void* stream);

/* Copy of `bytes` from d_src to both d_dst0 and d_dst1 (multiples of 16; 16-byte aligned,
 * non-overlapping): one byte read per two written, the HBM mix of an F stage that turns 4-byte
 * input samples into 8-byte channelised ones, so its rate is the streaming reference for that
 * kernel.  Errors: EINVAL, EDEVICE. */
int cobalt_device_fanout(void* d_dst0, void* d_dst1, const void* d_src, size_t bytes, void* stream);

/* Dense MFMA rate probe on the current device: `workgroups` workgroups of 256 threads (four
 * waves; two workgroups fit a CU) each run `iterations` rounds of eight independent
 * 32x32 MFMAs on register operands (x_mode COBALT_X_FP16_SPLIT: v_mfma_f32_32x32x16_f16,
 * 32768 flop each; COBALT_X_INT8: v_mfma_i32_32x32x32_i8, 65536 ops each), so the launch does
 * workgroups * 4 * iterations * 8 MFMAs.  Timed by the caller, it gives the MFMA rate the chip
 * sustains at the clock it holds under that load, next to which kernel rates can be read (a
 * readiness check, as the paper's operational scripts, sec. 8).  d_sink: device float
 * [workgroups * 256]; every element receives iterations * K (K = 16 FP16, 32 int8), or -1 if
 * a thread's accumulators disagree.  Errors: EINVAL (mode, iterations outside 1 .. 2^19,
 * workgroups outside 1 .. 2^20, NULL or misaligned sink), EDEVICE. */
int cobalt_mfma_probe(int32_t x_mode, int64_t iterations, int32_t workgroups, float* d_sink, void* stream);

/* ---- streaming service --------------------------------------------------------------
 * ~1 s blocks from several concurrent observations (the paper's correlator serves several
 * observations at once, each with its own station and subband set, sec. 7.1-7.3).
 *  - Memory: the service allocates its HBM budget once, as one device arena, and gives each
 *    observation a contiguous range of it for its working set: the plan workspace
 *    (cobalt_estimate_bytes), one device input block and one visibility buffer, each rounded
 *    up to 256 bytes.  Closing an observation returns its range (the paper allocates its
 *    buffers once and recycles them through pools of free blocks, sec. 7.1).
 *  - Admission: an observation that fits is admitted at once; one that does not fit yet
 *    waits, in arrival order, and is admitted as soon as closes free enough of the arena.
 *    Its blocks may be submitted meanwhile (they queue up to queue_depth).
 *  - Continuous batching: n_slots worker threads, each with its own stream, take the next
 *    queued block of any admitted observation that has no block running, so blocks of
 *    different observations overlap on the device; blocks of one observation run in arrival
 *    order, one at a time (the FIR history carries over).
 *  - Overload: a full FIFO drops the new block (COBALT_EBUSY) instead of stalling the
 *    producer, as the paper's pipeline drops data rather than wait (sec. 7.2).
 *  - Latency = submit -> the block's visibilities are back in host memory.
 *  - Host calls never hold the service's lock across a HIP call. */
typedef struct cobalt_service cobalt_service;

typedef struct cobalt_service_stats {
    int64_t submitted, completed, dropped, late;   /* late: latency > deadline; dropped: full
                                                      FIFO, or closed before admission     */
    double  p50_latency_s, p99_latency_s, max_latency_s;
    int64_t hbm_used_bytes, hbm_budget_bytes;      /* arena ranges held / arena size       */
    int64_t obs_admitted, obs_pending;             /* open observations by state           */
} cobalt_service_stats;

#define COBALT_OBS_PENDING   0   /* waiting for enough of the arena to be free             */
#define COBALT_OBS_ADMITTED  1
#define COBALT_OBS_CLOSED    2
#define COBALT_OBS_FAILED    3   /* admission failed (its plan could not be created)       */

/* Service on the current device: allocates the budget (rounded down to 256 bytes) as one
 * arena, creates `n_slots` streams (1..64) and as many worker threads; per-observation FIFOs
 * of `queue_depth` blocks; latency deadline in seconds.  Errors: EINVAL, ENOMEM (the arena),
 * EDEVICE. */
int cobalt_service_create(size_t hbm_budget_bytes, int n_slots, int queue_depth, double deadline_s,
                          cobalt_service** out);

/* Open an observation with setting cfg (host tables copied).  COBALT_OK: *obs_id identifies
 * it and it is either admitted or waiting for admission (cobalt_service_query tells which).
 * Errors: EINVAL, EUNSUPPORTED, EOVERFLOW (as cobalt_plan_create); ENOMEM when its working
 * set exceeds the whole budget (nothing is allocated); EDEVICE or ENOMEM when its plan could
 * not be created in an arena range that was free. */
int cobalt_service_open(cobalt_service* svc, const cobalt_config* cfg, int* obs_id);

/* *state = COBALT_OBS_PENDING / ADMITTED / CLOSED / FAILED (for FAILED,
 * cobalt_service_last_error() gives the reason).  Errors: EINVAL. */
int cobalt_service_query(cobalt_service* svc, int obs_id, int* state);

/* Queue one block: h_block host input ([S][P][SB][N] samples of the setting's type, S*2*SB*N
 * samples; pinned memory lets the copy run asynchronously), h_delays [S][2] (copied), h_vis
 * host output ([SB][C][B][4] complex visibilities, SB*C*B*32 bytes).  The library cannot
 * check the host buffers' sizes: they must hold at least these many bytes and stay valid
 * until cobalt_service_wait returns for *ticket.  A full FIFO drops the block: COBALT_EBUSY
 * with *ticket = -1.  Errors: EINVAL (unknown or closed observation), EBUSY, EDEVICE (the
 * observation's admission failed). */
int cobalt_service_submit(cobalt_service* svc, int obs_id, const void* h_block, const double* h_delays,
                          void* h_vis, int64_t* ticket);

/* Block until `ticket` has completed; *latency_s (may be NULL) = submit -> completion.  Each
 * ticket can be waited once.  Returns the block's own result: COBALT_OK, EBUSY (dropped
 * because its observation was closed before admission), EDEVICE (a device error while it
 * ran), or EINVAL (unknown ticket). */
int cobalt_service_wait(cobalt_service* svc, int64_t ticket, double* latency_s);

/* Stop (1) or resume (0) dispatching blocks; queued blocks stay queued (tests force full
 * FIFOs).  Admission continues while paused. */
int cobalt_service_pause(cobalt_service* svc, int paused);

/* Counters and latency percentiles over all completed blocks. */
int cobalt_service_get_stats(cobalt_service* svc, cobalt_service_stats* out);

/* Finish the observation's queued blocks (an observation still waiting for admission drops
 * them instead), then free its plan and return its arena range; waiting observations that
 * now fit are admitted. */
int cobalt_service_close(cobalt_service* svc, int obs_id);

/* Finish all queued blocks of admitted observations (blocks of observations still waiting
 * for admission are dropped), stop the workers and free everything.  Every cobalt_service_wait
 * must have returned first.  NULL is a no-op. */
int cobalt_service_destroy(cobalt_service* svc);

/* Message for the last service error on this host thread. */
const char* cobalt_service_last_error(void);

/* cobalt_correlate without a plan, for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid allocation): one block of
 * the full FX chain for setting cfg, allocating nothing.  Its intermediate data (the
 * channelised block between the F and X stages, the tables, a zero or discarded history)
 * live in a fixed scratch array of 256 MiB that every GPU the library runs on holds for the
 * life of the process; settings whose channelised block and tables exceed it are refused
 * (EUNSUPPORTED: use a plan).  The FIR history is the caller's: d_hist_in holds the
 * (T-1)*C samples of each stream that precede the block ([S*P*SB][(T-1)*C] samples of the
 * input type, stream (s*P + p)*SB + sb; NULL = zeros, a first block) and d_hist_out
 * receives those that follow it (NULL = discarded); they must not be the same buffer.
 * Every call on one GPU uses that GPU's one scratch array: calls that overlap on the device
 * (on different streams, or from several host threads) race and must be ordered by the
 * caller.  Host arrays (cfg tables, h_delays [S][2]) may be reused as soon as the call
 * returns.  samples_per_block must be > 0.  Errors: EINVAL, EUNSUPPORTED, EOVERFLOW, EDEVICE. */
int cobalt_correlate_noalloc(const cobalt_config* cfg, const void* d_in, const double* h_delays,
                             const void* d_hist_in, void* d_hist_out, void* d_vis, void* stream);

/* Wait for the plan's last call, then free everything it owns.  NULL is a no-op.
 * Errors: EDEVICE (the plan is freed anyway). */
int cobalt_plan_destroy(cobalt_plan* plan);

/* Message for the last error on this host thread ("" if none).  Never NULL. */
const char* cobalt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* COBALT_H */
