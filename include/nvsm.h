/*
 * nvsm.h - speckle-masking burst reconstruction on one AMD MI355X (gfx950).
 *
 * A burst of short-exposure frames goes in, one reconstructed image comes
 * out (Li et al., "High Performance Parallel Image Reconstruction for New
 * Vacuum Solar Telescope", Section 1: one burst of at least 100 short
 * exposures gives one image).  The burst is cut into partially overlapping
 * subimages (Section 3.2); for each, the mean power spectrum and the mean
 * bispectrum are accumulated over the frames, the Fourier modulus follows
 * from Labeyrie's relation (Eq. 1) with a speckle transfer function (STF)
 * table, the Fourier phase from the speckle-masking recursion (Sections 2
 * and 3.2), and the inverse transforms are merged into a mosaic
 * (Section 3.2).
 *
 * Conventions used throughout:
 *  - frames are [F][H][W] with x (the W axis) fastest; rows are
 *    row_pitch elements apart (W <= row_pitch <= 2^30 / N); one call takes at most
 *    F * (N/2 + 16) * N * 8 < 2^31 frames (26214 for N = 128, 87381 for
 *    N = 64; more gives NVSM_ERR_SHAPE);
 *  - a frequency u = (ux, uy) is stored at [uy mod N][ux mod N] of an
 *    N x N array ("DFT order");
 *  - the forward transform is exp(-2 pi i u.x / N), unnormalised;
 *  - W is the set of frequencies 0 < |w| <= u_cut with wy > 0 or
 *    (wy == 0 and wx > 0), ordered by |w|^2, then wy, then wx;
 *  - S is the set of bispectrum samples (w, v): w in W, 0 < |v| <= R,
 *    |v|^2 < |w|^2 and 0 < |w - v|^2 < |w|^2, ordered by w (as in W) then
 *    by (vy, vx);  B(w, v) = <I(w - v) I(v) conj I(w)> over frames;
 *  - patches are numbered row-major over the tile grid: row k starts at
 *    y = min(k * stride, H - N), column l at x = min(l * stride, W - N).
 *
 * Ownership: every buffer passed to a compute call is owned by the caller
 * and must stay valid until the work on `stream` has finished.  Device
 * buffers are device pointers on the context's device.  The context owns
 * only small constant tables (index sets, twiddles, work lists) that it
 * builds and uploads the first time a parameter set is used (or in
 * nvsm_prepare); compute calls allocate no device memory after that.
 *
 * Errors: every call returns an nvsm_status.  Arguments are validated
 * before anything is launched; a failed call has launched nothing.  Device
 * faults surface at the caller's next synchronisation.  Calls are
 * asynchronous on `stream` (a hipStream_t; NULL = the default stream).
 * A context is not thread-safe: use one per host thread.
 */
#ifndef NVSM_H
#define NVSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NVSM_OK = 0,
    NVSM_ERR_INVALID_ARG = -1,   /* null pointer, bad enum, bad parameter   */
    NVSM_ERR_SHAPE = -2,         /* sizes inconsistent with the parameters  */
    NVSM_ERR_WORKSPACE = -3,     /* workspace smaller than nvsm_plan says   */
    NVSM_ERR_OOM = -4,           /* host or device allocation failed        */
    NVSM_ERR_HIP = -5,           /* a HIP runtime call or launch failed     */
    NVSM_ERR_NOT_IMPLEMENTED = -6
} nvsm_status;

typedef enum { NVSM_U16 = 0, NVSM_F32 = 1 } nvsm_dtype;

typedef struct nvsm_context nvsm_context;

/* Reconstruction parameters.  nvsm_default_params fills the defaults. */
typedef struct {
    int32_t patch;        /* N, the subimage size: 64 or 128                */
    int32_t stride;       /* tile step, 1..N (default N/2: 50 % overlap)    */
    int32_t u_cut;        /* largest |w| reconstructed, < N/2 (default N/2-1) */
    int32_t v_radius;     /* R, largest |v| in the bispectrum, 1..16, < u_cut */
    int32_t window;       /* 0 none, 1 periodic Hann taper (default 1)      */
    int32_t phase_method; /* 0 recursive speckle-masking solve; 1 the same, then
                           * lsq_iters least-squares refinement steps      */
    int32_t noise_bias;   /* 0 off; 1 subtract the mean power beyond |u| > N/2+2
                           * in the solve; 2 photon-noise model (see
                           * nvsm_accumulate), gain photons_per_adu       */
    int32_t filter;       /* 0 none, 1 diffraction-limited OTF of the pupil  */
    double  stf_floor;    /* modulus 0 where STF < stf_floor (default 1e-6) */
    int32_t lsq_iters;    /* refinement steps for phase_method 1, 1..10000 (default 10) */
    int32_t reserved;     /* 0                                              */
    double  photons_per_adu; /* G for noise_bias 2: photons per unit of pixel
                           * value, finite and > 0 (default 1: frames in
                           * photon counts)                                 */
} nvsm_params;

/* Sizes derived from parameters and a burst shape (nvsm_plan). */
typedef struct {
    int32_t patches_y, patches_x; /* tile grid                              */
    int64_t patches;              /* patches_y * patches_x                  */
    int64_t w_count;              /* |W|                                    */
    int64_t s_count;              /* |S|                                    */
    int32_t shells;               /* distinct |w|^2 in W                    */
    int32_t frame_chunks;         /* frame groups of the accumulation       */
    size_t  ws_accumulate;        /* workspace bytes for nvsm_accumulate    */
    size_t  ws_solve;             /* workspace bytes for nvsm_solve         */
    size_t  ws_synthesize;        /* workspace bytes for nvsm_synthesize    */
    size_t  ws_reconstruct;       /* workspace bytes for nvsm_reconstruct   */
} nvsm_plan_info;

/* Context on HIP device `hip_device`.  *out is NULL on failure. */
nvsm_status nvsm_create(int hip_device, nvsm_context **out);
/* Frees the context and its tables (waits for nothing: synchronise first). */
void nvsm_destroy(nvsm_context *ctx);
/* Static text for a status code. */
const char *nvsm_status_string(nvsm_status s);
/* Text describing the context's last failure ("" if none). */
const char *nvsm_last_error(const nvsm_context *ctx);

/* Defaults for patch size N (64 or 128): stride N/2, u_cut N/2-1, R 10,
 * Hann window, recursive phase (10 refinement steps if phase_method is set
 * to 1), no noise bias (photons_per_adu 1), no filter, floor 1e-6. */
nvsm_status nvsm_default_params(int32_t patch, nvsm_params *out);

/* Validates params against an H x W x F burst and fills *out.  Host only. */
nvsm_status nvsm_plan(const nvsm_params *p, int32_t H, int32_t W, int32_t F,
                      nvsm_plan_info *out);

/* The set W in its storage order: w[i*2 + 0] = wx, w[i*2 + 1] = wy.
 * Host buffer of 2*w_count int32; w_count must equal |W|.  Host only. */
nvsm_status nvsm_w_index(const nvsm_params *p, int32_t *w, int64_t w_count);

/* The set S in its storage order: wv[i*4 + 0..3] = (wx, wy, vx, vy).
 * Host buffer of 4*s_count int32; s_count must equal |S|.  Host only. */
nvsm_status nvsm_bispectrum_index(const nvsm_params *p, int32_t *wv, int64_t s_count);

/* Builds and uploads the context's tables for `p` (synchronous).  Optional:
 * the compute calls do it on first use of a parameter set. */
nvsm_status nvsm_prepare(nvsm_context *ctx, const nvsm_params *p);

/* Accumulation over the burst (Eq. 1 numerator and the speckle-masking
 * bispectrum).  For every patch k, with p_f the N x N cut of frame f and
 * t the taper: mu_f = sum(t p_f) / sum(t), I_f = FFT2((p_f - mu_f) t).
 * Outputs (device, caller-owned):
 *   power     [P][N][N] float   <|I_f(u)|^2>, DFT order
 *   mean_spec [P][2][2] float   <I_f(1,0)> and <I_f(0,1)> as (re, im)
 *   mu        [P]       float   <mu_f>
 *   bispec    [P][|S|][2] float <I_f(w-v) I_f(v) conj I_f(w)> in S order,
 *             or NULL to skip the bispectrum.
 * frames: device [F][H][row_pitch] of uint16 or float32.
 * Arithmetic: FP32; sums over frames use compensated (Kahan) summation.
 * noise_bias 2 (photon noise; the paper gives no noise model): pixel values
 * are Poisson photon counts over G = photons_per_adu.  With
 * Q_f = FFT2(t^2 p_f) / G, C(u) = <conj I_f(u) Q_f(u)>, q0 = <sum t^2 p_f> / G
 * and T = <sum t^3 p_f> / G^2, power is returned as <|I_f|^2> - q0 and
 * bispec as the mean minus C(w) + conj C(v) + conj C(w-v) - 2T: the noise
 * terms in expectation wherever the taper's transform vanishes at w, v and
 * w - v (for the Hann taper: each has a component of modulus >= 2; with no
 * taper: all of them), in the manner of the photon-counting corrections of
 * speckle interferometry and speckle masking.  The streaming calls carry
 * these terms too (their sums run over the groups like the others'). */
nvsm_status nvsm_accumulate(nvsm_context *ctx, const nvsm_params *p,
                            const void *frames, nvsm_dtype dtype, int32_t F,
                            int32_t H, int32_t W, int64_t row_pitch,
                            float *power, float *mean_spec, float *mu, float *bispec,
                            void *workspace, size_t workspace_bytes, void *stream);

/* Modulus and phase per patch, FP64 (Eq. 1; speckle-masking recursion).
 *   amp[k][i]    = sqrt(max(power(w_i) - n, 0) / stf(w_i)), 0 where
 *                  stf(w_i) < stf_floor; n is the corner noise level
 *                  with noise_bias 1, else 0 (noise_bias 2 corrects power
 *                  in the accumulation).  double [P][|W|].
 *   phasor[k][i] = e(w_i) (re, im), double [P][|W|][2]: e(1,0), e(0,1) are
 *                  the unit phasors of mean_spec, and every other w takes the
 *                  phase of sum_v e(w-v) e(v) conj B(w,v) over its samples,
 *                  in increasing |w| (e(-u) = conj e(u); 1 when the sum is 0).
 *   phase_method 1 then refines the phasors by least squares: lsq_iters
 *                  steps, each moving every e(u) but the two seeds halfway
 *                  (e' = unit(unit(g) + e)) to the unit of
 *                    g(u) = sum over the samples holding u of the derivative
 *                           of sum_S Re[e(w-v) e(v) conj e(w) conj B] by
 *                           conj e(u),
 *                  all from the previous step's phasors (Jacobi). 
 * Inputs: power, mean_spec, bispec as produced by nvsm_accumulate for
 * `patches` patches; stf: device double [N][N] in DFT order. */
nvsm_status nvsm_solve(nvsm_context *ctx, const nvsm_params *p, int64_t patches,
                       const float *power, const float *mean_spec, const float *bispec,
                       const double *stf, double *amp, double *phasor,
                       void *workspace, size_t workspace_bytes, void *stream);

/* Inverse transform and mosaic (Section 3.2).  For each patch the spectrum
 * filter(w) amp e(w) on W (conjugate at -w, 0 elsewhere) is transformed
 * back (FP32), mu * taper is added, and the mosaic is
 *   out(x) = sum_k r_k(x - o_k) / sum_k t(x - o_k)  (0 where the sum < 1e-3).
 * patches_out: device float [P][N][N] to keep the subimages, or NULL (then
 * the workspace holds them).  out: device float [H][W]. */
nvsm_status nvsm_synthesize(nvsm_context *ctx, const nvsm_params *p, int32_t H, int32_t W,
                            const double *amp, const double *phasor, const float *mu,
                            float *patches_out, float *out,
                            void *workspace, size_t workspace_bytes, void *stream);

/* The whole path: frames (device) in, image out (device float [H][W]).
 * Equivalent to accumulate + solve + synthesize with all intermediates in
 * the workspace (nvsm_plan_info.ws_reconstruct bytes).  When the call
 * returns (and likewise after nvsm_reconstruct_batch, for the P patches of
 * its last launch group, numbered burst by burst) the workspace starts with
 * the intermediates in this order, each at a 256-byte aligned offset:
 * power float [P][N][N], mean_spec float [P][2][2], mu float [P],
 * bispec float [P][|S|][2], amp double [P][|W|], phasor double [P][|W|][2],
 * subimages float [P][N][N] (each as nvsm_accumulate, nvsm_solve and
 * nvsm_synthesize define them). */
nvsm_status nvsm_reconstruct(nvsm_context *ctx, const nvsm_params *p,
                             const void *frames, nvsm_dtype dtype, int32_t F,
                             int32_t H, int32_t W, int64_t row_pitch,
                             const double *stf, float *out,
                             void *workspace, size_t workspace_bytes, void *stream);

/* nvsm_reconstruct for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same path and the same result bit for bit, with the
 * workspace taken from a fixed array in the library's device data instead of
 * a caller buffer.  The array holds 256 MiB on each GPU the library runs on
 * (found once per device by nvsm_create, kept until the process ends): a
 * burst whose nvsm_plan_info.ws_reconstruct exceeds that gives
 * NVSM_ERR_WORKSPACE and launches nothing.  The parameter set's tables must
 * exist first (nvsm_prepare, or an earlier compute call with p), else
 * NVSM_ERR_INVALID_ARG; the call then allocates nothing and records no
 * stage-timing events.  Every call on one GPU shares that GPU's array (it
 * keeps the last call's intermediates; nothing in it needs clearing between
 * calls): calls that overlap on one GPU, on different streams or from
 * different contexts, race and give wrong results.  Order them. */
nvsm_status nvsm_reconstruct_noalloc(nvsm_context *ctx, const nvsm_params *p,
                                     const void *frames, nvsm_dtype dtype, int32_t F,
                                     int32_t H, int32_t W, int64_t row_pitch,
                                     const double *stf, float *out, void *stream);

/* One burst of a batch.  frames: device [F][H][row_pitch] pixels of the
 * batch's dtype; stf: device double [N][N] (DFT order) for this burst's
 * seeing; out: device float [H][W].  All caller-owned. */
typedef struct nvsm_burst {
    const void *frames;
    int32_t F, H, W;
    int64_t row_pitch;
    const double *stf;
    float *out;
} nvsm_burst;

/* Workspace for nvsm_reconstruct_batch on these bursts (host call, no
 * device access; pointers may be NULL): *ws_min is enough to run them one
 * burst per launch group, *ws_all to run up to 16 per group.  Any size in
 * between works; larger groups share launches. */
nvsm_status nvsm_batch_plan(const nvsm_params *p, const nvsm_burst *bursts, int32_t n,
                            size_t *ws_min, size_t *ws_all);

/* The whole path (as nvsm_reconstruct) for n bursts of uneven shape and
 * frame count that share the parameters p and the dtype.  The bursts are
 * taken in order in groups of at most 16 whose intermediates fit in the
 * workspace; each group runs as one launch per stage over all patches of
 * its bursts (workgroups find their burst from the patch and workgroup
 * numbering), so small bursts fill the GPU together.  Each image equals
 * the one nvsm_reconstruct gives for that burst alone, bit for bit: every
 * value is computed by the same arithmetic in the same order.  Launches go
 * to `stream` and allocate nothing, so the call can be captured in a HIP
 * graph once the plan exists (nvsm_prepare). */
nvsm_status nvsm_reconstruct_batch(nvsm_context *ctx, const nvsm_params *p, nvsm_dtype dtype,
                                   const nvsm_burst *bursts, int32_t n,
                                   void *workspace, size_t workspace_bytes, void *stream);

/* Streaming accumulation of one burst whose frames arrive over time (for
 * a serving loop).  Two caller-owned device buffers:
 *   state (one per burst in flight): the running compensated (Kahan)
 *     sums, (sum, compensation) pairs, of the bispectrum terms, kept in the
 *     kernel's own order so that every pass over them is coalesced, and of
 *     the power spectrum, mean spectrum and mean level (with noise_bias 2
 *     also those of the photon-noise terms C, q0 and T);
 *   ws (one per stream of calls): scratch for one group of frames and the
 *     final buffers.  After the last group its first P * |S| * 8 bytes
 *     hold the bispectrum means, float [P][|S|][2] in S order, as
 *     nvsm_accumulate writes them.
 *   nvsm_stream_plan: state and ws bytes for an H x W burst added in groups
 *     of up to group_frames frames (host call).
 *   nvsm_stream_add: ingests G frames (device [G][H][row_pitch]) and adds
 *     their terms to the running sums.  frames_before = frames of this
 *     burst already added (0 for the first group, which starts the sums
 *     from zero whatever the state holds); total_frames = 0 except for the
 *     last group, where it is the burst's frame count (= frames_before + G)
 *     and the call writes the means over all frames into ws.  Within a
 *     group frames are summed in blocks as usual; each group's sums are
 *     folded into the running pairs.  One group of all F frames gives
 *     exactly nvsm_accumulate's values (noise_bias 2: the last group
 *     subtracts the photon-noise terms' means over all frames).
 *   nvsm_stream_finish: modulus, phase, subimages and mosaic (as
 *     nvsm_solve + nvsm_synthesize) from ws after the last group, into out
 *     [H][W].
 * Calls on one state or one ws must be ordered (same stream or events);
 * different states are independent, so bursts of several channels may run
 * on several streams, each with its own ws.  These calls always run 16
 * slots per wave (see nvsm_autotune), so the state's layout does not depend
 * on the launch choice, which may change between the calls of a burst.
 * None of these calls allocates device memory once the plan exists. */
nvsm_status nvsm_stream_plan(const nvsm_params *p, int32_t H, int32_t W, int32_t group_frames,
                             size_t *state_bytes, size_t *ws_bytes);
nvsm_status nvsm_stream_add(nvsm_context *ctx, const nvsm_params *p, const void *frames,
                            nvsm_dtype dtype, int32_t G, int32_t H, int32_t W, int64_t row_pitch,
                            int32_t frames_before, int32_t total_frames, void *state,
                            size_t state_bytes, void *ws, size_t ws_bytes, void *stream);
nvsm_status nvsm_stream_finish(nvsm_context *ctx, const nvsm_params *p, int32_t H, int32_t W,
                               const double *stf, float *out, void *ws, size_t ws_bytes,
                               void *stream);

/* Launch tuning for the bispectrum stage of p's plan.  The candidates are
 * implementations of the same arithmetic in the same order, so every
 * output is identical whichever is chosen; only the time differs:
 *   slots per wave: 16 or 24 v values per wave of a work item;
 *   form: 0 one workgroup per work item, 1 a persistent grid of resident
 *         workgroups taking items from per-XCD work queues (their counters
 *         live in the call's own workspace, so calls with different
 *         workspaces may run concurrently on different streams).
 * The streaming calls keep 16 slots per wave whatever the choice (their
 * running sums are stored in that kernel's lane order) and use its form.
 * nvsm_autotune runs the ingest once on the given burst (device frames,
 * as for nvsm_reconstruct, with a workspace of ws_reconstruct bytes), then
 * times the bispectrum launch of each candidate with HIP events and keeps
 * the fastest for p (it waits for the stream).  *slots_out and *form_out
 * (may be NULL) receive the choice.  nvsm_set_launch sets a choice
 * directly.  Without either, calls use 16 slots and form 0. */
nvsm_status nvsm_autotune(nvsm_context *ctx, const nvsm_params *p,
                          const void *frames, nvsm_dtype dtype, int32_t F,
                          int32_t H, int32_t W, int64_t row_pitch,
                          void *workspace, size_t workspace_bytes, void *stream,
                          int32_t *slots_out, int32_t *form_out);
nvsm_status nvsm_set_launch(nvsm_context *ctx, const nvsm_params *p, int32_t slots, int32_t form);

/* The v radius R of a schedule (one R per patch size and burst shape, e.g.
 * per class of a batch), chosen on the caller's burst at a stated accuracy.
 * R sets how many bispectrum samples the phase recursion averages (Sections
 * 2 and 3.2; the paper does not state its domain); the work grows as R^2.
 * On the patches of the burst's central crop (at most 512 x 512 px) the
 * path runs at R = r_max and then at r_min, r_min + 1, ... (p otherwise),
 * and stops at the first R whose phases agree with those at r_max within
 * tol radians: the weighted RMS of the wrapped phase difference over W and
 * the crop's patches, sqrt(sum P dphi^2 / sum P), P(w) the mean power
 * spectrum of the frames less its noise floor (the mean power where
 * |u| > N/2 + 2, per patch), 0 where below it: the frequencies the frames
 * carry strongly count most and those at the floor, whose phases are noise,
 * not at all (the STF-divided modulus would weight the noise-dominated high
 * frequencies most).  *r_out receives that R (r_max when none is closer);
 * err (host double [r_max - r_min + 1], or NULL) the measure of every R
 * tried (0 at r_max, NaN where not run).  frames, stf as nvsm_reconstruct;
 * workspace: nvsm_tune_radius_plan bytes.  Builds the tables of every R it
 * runs; waits for `stream` (copies the phases to the host). */
nvsm_status nvsm_tune_radius_plan(const nvsm_params *p, int32_t H, int32_t W, int32_t F, int32_t r_max,
                                  size_t *ws_bytes);
nvsm_status nvsm_tune_radius(nvsm_context *ctx, const nvsm_params *p, const void *frames, nvsm_dtype dtype,
                             int32_t F, int32_t H, int32_t W, int64_t row_pitch, const double *stf,
                             int32_t r_min, int32_t r_max, double tol, void *workspace,
                             size_t workspace_bytes, void *stream, int32_t *r_out, double *err);

/* Model speckle transfer function (the STF of Eq. 1 chosen by the seeing
 * D/r0, Sections 2 and 3.2; the paper gives no model, so this is a reading):
 * a Monte Carlo mean over `screens` Kolmogorov phase screens (phase spectrum
 * 0.023 r0^(-5/3) f^(-11/3), FFT method plus three subharmonic levels of Lane,
 * Glindemann and Dainty 1992) across a circular pupil of diameter N/2 px in
 * the N x N patch grid (r0 = (N/2) / d_over_r0 px), so the PSF
 * |FFT2(pupil exp(i phi))|^2 is Nyquist sampled on the patch grid; per screen
 * OTF = FFT2(PSF) / OTF(0).
 *   stf      device double [N][N], DFT order: <|OTF|^2> (1 at u = 0); the
 *            table nvsm_solve and nvsm_reconstruct take.
 *   mean_otf device double [N][N][2] (re, im) <OTF>, or NULL.
 * Random numbers: Philox4x32-10 with key (seed mod 2^32, seed div 2^32) and
 * counter (screen pair, word, 0, 0); the same seed gives the same table.
 * screens: even, 2 .. 2^24 (two screens per transform); d_over_r0 in
 * (0, 1000].  workspace: nvsm_model_stf_plan bytes of partial sums, owned by
 * the caller; asynchronous on `stream`. */
nvsm_status nvsm_model_stf_plan(const nvsm_params *p, int32_t screens, size_t *ws_bytes);
nvsm_status nvsm_model_stf(nvsm_context *ctx, const nvsm_params *p, double d_over_r0, int32_t screens,
                           uint64_t seed, double *stf, double *mean_otf, void *workspace,
                           size_t workspace_bytes, void *stream);

/* Seeing estimate by the spectral ratio (Sections 2 and 3.2: the paper
 * finds r0 from the burst on non-overlapping subimage cubes, averages it and
 * chooses the model STF by it; it gives no formulas, so this is a reading).
 * Cubes: the full N x N tiles of the frame on a grid of step N.  Per cube,
 * with the taper and mean removal of nvsm_accumulate, m = <I_f> and
 * P = <|I_f|^2>: eps(u) = (|m|^2 - P/F) / (P (1 - 1/F)), averaged over the
 * annuli q - 1/2 <= |u| < q + 1/2 (q = 1..bins).  Model curves, on the grid
 * D/r0 = min (max/min)^(j/(points-1)): rho = |<OTF>|^2 / <|OTF|^2> of the
 * nvsm_model_stf Monte Carlo (model point j is Philox counter word 2 = j),
 * seen through the taper as sum_k |w(k)|^2 P(u-k) rho(u-k) / sum_k
 * |w(k)|^2 P(u-k) (|w|^2 = 1/4, 1/16 per axis at offsets 0, +-1; only k = 0
 * without a taper), averaged over the same annuli.  A cube's D/r0 minimises
 * the squared distance of the curves (first minimum, then the vertex of the
 * parabola through it and its neighbours, in grid index); the burst's is
 * 1 / <1 / (D/r0)> over the cubes.
 *   d_over_r0 device double [1 + cubes]: the burst's value, then each cube's.
 *   stf       device double [N][N]: the model STF at the burst's value
 *             (nvsm_model_stf with counter word 2 = points), ready for
 *             nvsm_solve / nvsm_reconstruct.
 *   curves    device double [cubes][bins] ratio curves, or NULL.
 * F >= 2; H, W >= N.  workspace: nvsm_seeing_plan bytes.  Asynchronous on
 * `stream` (nothing is read back to the host). */
typedef struct {
    int32_t screens;        /* Monte Carlo screens per model point, even, 2..2^24 (default 1000) */
    int32_t points;         /* model points of the D/r0 grid, 3..256 (default 40) */
    double  d_over_r0_min;  /* grid ends, 0 < min < max <= 1000 (default 2, 50) */
    double  d_over_r0_max;
    int32_t bins;           /* annuli of the fit, 2..min(24, N/4) (default 12) */
    int32_t reserved;       /* 0 */
    uint64_t seed;          /* Philox key (default 1) */
} nvsm_seeing_params;
nvsm_status nvsm_seeing_default_params(nvsm_seeing_params *out);
nvsm_status nvsm_seeing_plan(const nvsm_params *p, const nvsm_seeing_params *sp, int32_t H, int32_t W, int32_t F,
                             size_t *ws_bytes, int32_t *cubes);
nvsm_status nvsm_seeing(nvsm_context *ctx, const nvsm_params *p, const nvsm_seeing_params *sp,
                        const void *frames, nvsm_dtype dtype, int32_t F, int32_t H, int32_t W,
                        int64_t row_pitch, double *d_over_r0, double *stf, double *curves,
                        void *workspace, size_t workspace_bytes, void *stream);

/* Stage timing with HIP events recorded on the call's stream around each
 * stage's kernels (off by default; recording adds no synchronisation).
 * Stages: 0 ingest (tile cut, taper, FFT, power and mean sums),
 * 1 bispectrum accumulation, 2 modulus and phase solve, 3 synthesis and
 * mosaic.  Enabling creates events on first use; 0 disables. */
nvsm_status nvsm_profile_enable(nvsm_context *ctx, int32_t enable);
/* Waits for every recorded stage, adds its elapsed milliseconds to ms[stage]
 * and its launch count to count[stage] (host arrays of n >= 4 entries), and
 * forgets the records. */
nvsm_status nvsm_profile_read(nvsm_context *ctx, double *ms, int64_t *count, int32_t n);

#ifdef __cplusplus
}
#endif
#endif /* NVSM_H */
