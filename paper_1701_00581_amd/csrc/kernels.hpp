// Launch interfaces of the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nvsm {

// One burst of a launch.  A launch covers up to MAX_BURSTS bursts that
// share the patch size and index sets; their patches are numbered
// consecutively (patch0), as are their ingest workgroups (ingest0), stored
// spectrum records (spec0, in records of one patch and frame) and output
// pixels (pix0).  The table travels by value in the kernel arguments.
constexpr int MAX_BURSTS = 16;
struct BurstDesc {
    const void *frames = nullptr;         // [F][H][pitch] pixels
    int64_t pitch = 0;                    // pixels per row
    int64_t spec0 = 0;                    // first stored spectrum record
    int64_t pix0 = 0;                     // first output pixel (mosaic)
    const double *stf = nullptr;          // [N][N]
    float *out = nullptr;                 // [H][W]
    int F = 0, H = 0, W = 0, ny = 0, nx = 0;
    int patch0 = 0, ingest0 = 0, pad = 0;
};
struct BurstTable {
    int nb = 0;
    int patches = 0;                      // total over the bursts
    int ingest_wgs = 0;                   // total ingest workgroups
    int pad = 0;
    int64_t pixels = 0;                   // total output pixels
    BurstDesc b[MAX_BURSTS];
};

struct IngestArgs {
    int N = 0;
    bool f32 = false;
    BurstTable bt;
    int stride = 0, chunk_frames = 0, window = 0;
    bool vec = false;                     // every burst allows 4-pixel vector loads
    float inv_wsum = 0.f;
    const float2 *twiddle = nullptr;
    const float *hann = nullptr;
    float2 *spectra = nullptr;            // [records][N/2 + 16][N], rows -16 .. N/2-1
    float *ppart = nullptr, *mpart = nullptr, *mupart = nullptr;   // per ingest workgroup
    float *power = nullptr, *mean_spec = nullptr, *mu = nullptr;   // per patch
    // streaming (one burst): 0 all frames at once; 1 add this frame group
    // to the running sums (from zero when stream_first); 2 add the last
    // group and write the means
    int stream_mode = 0, stream_first = 0;
    float2 *psc = nullptr, *msc = nullptr, *musc = nullptr;        // running (sum, compensation)
    float inv_total = 0.f;
};
hipError_t launch_ingest(const IngestArgs &a, hipStream_t st);

// Photon-noise terms (pixel values Poisson counts over a gain G).  Per patch
// and frame, with t the taper and I the spectrum of the ingest:
// Q = FFT2(t^2 p) / G, C(u) = conj I(u) Q(u), q0 = sum(t^2 p) / G,
// T = sum(t^3 p) / G^2.  launch_noise accumulates their means over the
// frames (the workgroups of the ingest grid, then one pass per patch that
// writes C in the record layout of the spectra and subtracts q0 from the
// power spectrum); the bispectrum launch then subtracts
// C(w) + conj C(v) + conj C(w - v) - 2T as it writes each mean.
struct NoiseArgs {
    IngestArgs in;                        // grid, frames, taper, power spectrum
    float inv_gain = 0.f;                 // 1 / G
    float2 *cpart = nullptr;              // [ingest wgs][N/2 + 1][N] sums of C over a frame group
    float *spart = nullptr;               // [ingest wgs][2] sums of q0 and T
    float2 *cgrid = nullptr;              // [P][N/2 + 16][N] mean C, record layout
    float *nbar = nullptr;                // [P][2] mean q0 and T
    // streaming (in.stream_mode 1 or 2, one burst): the group's sums go into
    // running (sum, compensation) pairs, from zero when in.stream_first; the
    // last group (mode 2) writes the means over in.inv_total frames
    float4 *csc = nullptr;                // [P][N/2 + 1][N] C: (sum re, sum im, comp re, comp im)
    float *ssc = nullptr;                 // [P][4] q0 and T: (sum, sum, comp, comp)
};
hipError_t launch_noise(const NoiseArgs &a, hipStream_t st);

// Seeing by the spectral ratio (see k_ingest.hip, k_stf.hip).
constexpr int RATIO_MAX_BINS = 24;        // annuli q = 1..bins
constexpr int RATIO_MAX_POINTS = 256;     // model points of the D/r0 grid
struct RatioArgs {
    int N = 0;
    bool f32 = false, vec = false;
    const void *frames = nullptr;         // [F][H][pitch]
    int F = 0, H = 0, cubes = 0, nx = 0, chunk_frames = 0, window = 0, B = 0;
    int64_t pitch = 0;
    float inv_wsum = 0.f;
    const float2 *twiddle = nullptr;
    const float *hann = nullptr;
    float *part = nullptr;                // [cubes * chunks][(B + 1)(2B + 1)][3]
};
hipError_t launch_ratio(const RatioArgs &a, hipStream_t st);
struct SeeingFitArgs {
    int N = 0, cubes = 0, nchunks = 0, F = 0, B = 0, Q = 0, J = 0, window = 0;
    double lo = 0.0, hi = 0.0;            // D/r0 grid lo (hi/lo)^(j/(J-1))
    const float *part = nullptr;          // from launch_ratio
    const double *tab_s = nullptr;        // [J][N][N] model <|OTF|^2>
    const double2 *tab_a = nullptr;       // [J][N][N] model <OTF>
    double *x = nullptr;                  // [1 + cubes]: burst, then per cube
    double *curves = nullptr;             // [cubes][Q] ratio curves, or null
};
hipError_t launch_seeing_fit(const SeeingFitArgs &a, hipStream_t st);

// Model speckle transfer function by Monte Carlo over Kolmogorov screens
// (see k_stf.hip): screens = 2 pairs; nwg workgroups each sum their pairs'
// <OTF> and <|OTF|^2> over the half plane into part_a / part_s; stf (and
// mean_otf if not null) receive the means over the full N x N grid (DFT
// order, FP64).
struct StfArgs {
    int N = 0, pairs = 0, nwg = 0;
    float amp = 0.f;                      // sqrt(0.023) r0^(-5/6) N^(5/6), r0 in px
    uint32_t k0 = 0, k1 = 0, stream = 0;  // Philox key and counter word 2
    const float2 *twiddle = nullptr;
    float2 *part_a = nullptr;             // [nwg][N/2 + 1][N]
    float *part_s = nullptr;              // [nwg][N/2 + 1][N]
    double *stf = nullptr;                // [N][N]
    double2 *mean_otf = nullptr;          // [N][N] or null
    const double *x_dev = nullptr;        // D/r0 in device memory (then amp is computed from it), or null
};
hipError_t launch_stf(const StfArgs &a, hipStream_t st);

// Zeroes bytes (a multiple of 16, 16-byte aligned) with a fill kernel.
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st);

// Accumulator handling of the bispectrum launch.  mode 0: the launch covers
// all frames and writes the mean.  mode 1: the launch adds a group of
// frames to running (sum, compensation) pairs kept between launches in the
// kernel's lane order (coalesced), starting from zero when first.  mode 2:
// as 1 for the last group, then writes the mean, (sum - comp) * inv_total,
// to the bispectrum array in S order.
// noise_c/noise_t (mode 0, or mode 2 of the streaming form): photon-noise
// terms to subtract from the mean, C per patch in the record layout of the
// spectra ([P][N/2 + 16][N]) and (q0, T) per patch (see NoiseArgs).
struct AccState {
    float2 *sum = nullptr, *comp = nullptr;   // [P * n_items * 4 * slots * 64]
    int mode = 0, first = 0, n_items = 0;
    float inv_total = 0.f;
    const float2 *noise_c = nullptr;
    const float *noise_t = nullptr;
};

struct BispecArgs {
    int N = 0;
    BurstTable bt;
    const float2 *spectra = nullptr;
    int n_items = 0, slots = 0;
    const int *items = nullptr, *group_xy = nullptr, *slot_v = nullptr, *out_idx = nullptr;
    float2 *bispec = nullptr;             // [P][|S|]
    int64_t s_count = 0;
    int form = 0;                         // 0: one workgroup per item, 1: persistent work queue
    int *queue = nullptr;                 // [8] counters for the work queue
    AccState acc;
};
hipError_t launch_bispec(const BispecArgs &a, hipStream_t st);

struct SolveArgs {
    int N = 0, nW = 0, max_sw = 0;
    BurstTable bt;                        // patches and the STF of each burst
    const int *woff = nullptr, *Wxy = nullptr;
    const int *w_slot = nullptr;          // LDS slot of each w's phasor
    const int *units = nullptr;           // phase-solve units (see plan.hpp)
    int n_units = 0;
    int n_inner = 0, ring = 0;            // phasor window (see plan.hpp)
    int zero_slot = 0;                    // window slot of the zero phasor
    const unsigned *code = nullptr;       // padded sample codes with LDS slots (solve_code)
    const float *power = nullptr, *mean_spec = nullptr;
    const float2 *bispec = nullptr;
    int64_t s_count = 0;
    double floor = 0;
    int noise_bias = 0;
    double *amp = nullptr;
    double2 *phasor = nullptr;
    // least-squares refinement (phase_method 1)
    int phase_method = 0, lsq_iters = 0;
    const unsigned *wcode = nullptr;      // sample codes with W indices
    const int *lsq_fin = nullptr;         // flushed prefix before each round (see plan.hpp)
    SolveArgs() = default;
    SolveArgs(const SolveArgs &o, int method) : SolveArgs(o) { phase_method = method; }
};
hipError_t launch_solve(const SolveArgs &a, hipStream_t st);

struct SynthArgs {
    int N = 0, nW = 0, window = 0;
    BurstTable bt;                        // patches, tilings and output images
    const int *Wxy = nullptr;
    const double *amp = nullptr;
    const double2 *phasor = nullptr;
    const float *filt = nullptr;          // nullptr = no filter
    const float *mu = nullptr, *hann = nullptr;
    const float2 *twiddle = nullptr;
    float *patch_buf = nullptr;           // [P][N][N]
    int stride = 0;
    bool mosaic = true;
};

// The burst of workgroup or item index L, given each burst's first index.
template <typename Get>
__device__ __forceinline__ int burst_of(const BurstTable &bt, int64_t L, Get first) {
    int b = 0;
    while (b + 1 < bt.nb && L >= first(bt.b[b + 1])) ++b;
    return b;
}
hipError_t launch_synth(const SynthArgs &a, hipStream_t st);

}  // namespace nvsm
