// Launch interfaces of the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nvsm {

struct IngestArgs {
    int N = 0;
    bool f32 = false;
    const void *frames = nullptr;
    int F = 0, H = 0, W = 0;
    int64_t pitch = 0;
    int patches = 0, nx = 0, stride = 0, chunk_frames = 0, nchunks = 0, window = 0;
    float inv_wsum = 0.f;
    const float2 *twiddle = nullptr;
    const float *hann = nullptr;
    float2 *spectra = nullptr;            // [P][F][N/2 + 16][N], rows -16 .. N/2-1
    float *ppart = nullptr, *mpart = nullptr, *mupart = nullptr;
    float *power = nullptr, *mean_spec = nullptr, *mu = nullptr;
};
hipError_t launch_ingest(const IngestArgs &a, hipStream_t st);

struct BispecArgs {
    int N = 0;
    const float2 *spectra = nullptr;
    int F = 0, patches = 0, n_items = 0, slots = 0;
    const int *items = nullptr, *group_xy = nullptr, *slot_v = nullptr, *out_idx = nullptr;
    float2 *bispec = nullptr;             // [P][|S|]
    int64_t s_count = 0;
};
hipError_t launch_bispec(const BispecArgs &a, hipStream_t st);

struct SolveArgs {
    int N = 0, patches = 0, nW = 0, nshell = 0, max_sw = 0;
    const int *shell_wb = nullptr, *woff = nullptr, *Wxy = nullptr;
    const int *w_slot = nullptr;          // LDS slot of each w's phasor
    int n_inner = 0, ring = 0;            // phasor window (see plan.hpp)
    const unsigned *code = nullptr;       // sample codes with LDS slots
    const float *power = nullptr, *mean_spec = nullptr;
    const float2 *bispec = nullptr;
    int64_t s_count = 0;
    const double *stf = nullptr;
    double floor = 0;
    int noise_bias = 0;
    double *amp = nullptr;
    double2 *phasor = nullptr;
};
hipError_t launch_solve(const SolveArgs &a, hipStream_t st);

struct SynthArgs {
    int N = 0, patches = 0, nW = 0, window = 0;
    const int *Wxy = nullptr;
    const double *amp = nullptr;
    const double2 *phasor = nullptr;
    const float *filt = nullptr;          // nullptr = no filter
    const float *mu = nullptr, *hann = nullptr;
    const float2 *twiddle = nullptr;
    float *patch_buf = nullptr;           // [P][N][N]
    int H = 0, W = 0, ny = 0, nx = 0, stride = 0;
    float *out = nullptr;                 // [H][W]
};
hipError_t launch_synth(const SynthArgs &a, hipStream_t st);

}  // namespace nvsm
