// Inverse transform of modulus and phase, and the mosaic (Section 3.2).
//
// k_synth: one workgroup per patch builds the Hermitian spectrum
// filter(w) |O(w)| e(w) on W in LDS and inverts it with the forward FFT:
// Re IFFT(X) = Re FFT(conj X) / N^2.  The mean level removed at ingest is
// put back under the taper.
// k_mosaic: one thread per output pixel of the bursts of the launch gathers
// the (at most 3 x 3) subimages covering it, out = sum r_k / sum taper_k
// (0 where < 1e-3).
#include "device_common.hpp"
#include "kernels.hpp"

namespace nvsm {

namespace {

constexpr int NT = 256;

template <int N>
__global__ __launch_bounds__(NT) void k_synth(int nW, const int *__restrict__ Wxy,
                                              const double *__restrict__ amp,
                                              const double2 *__restrict__ phasor,
                                              const float *__restrict__ filt, const float *__restrict__ mu,
                                              int window, const float *__restrict__ hann,
                                              const float2 *__restrict__ twiddle,
                                              float *__restrict__ patches) {
    constexpr int P = LdsPitch<N>::v;
    __shared__ float2 z[N * P];
    __shared__ float2 tw[N];
    __shared__ float hw[N];
    const int patch = blockIdx.x, tid = threadIdx.x;
    for (int i = tid; i < N; i += NT) {
        tw[i] = twiddle[i];
        hw[i] = window ? hann[i] : 1.0f;
    }
    for (int j = tid; j < N * P; j += NT) z[j] = make_float2(0.f, 0.f);
    __syncthreads();
    for (int i = tid; i < nW; i += NT) {
        const int wx = Wxy[2 * i], wy = Wxy[2 * i + 1];
        const float a = (float)amp[(size_t)patch * nW + i] * (filt ? filt[i] : 1.0f);
        const double2 e = phasor[(size_t)patch * nW + i];
        const float2 v = make_float2(a * (float)e.x, a * (float)e.y);
        z[(wy & (N - 1)) * P + (wx & (N - 1))] = conjf2(v);
        z[((-wy) & (N - 1)) * P + ((-wx) & (N - 1))] = v;
    }
    __syncthreads();
    fft2d_lds<N, NT>(z, tw);
    const float m = mu[patch];
    constexpr float inv = 1.0f / (float)(N * N);
    float *out = patches + (size_t)patch * N * N;
    for (int j = tid; j < N * N; j += NT) {
        const int y = j / N, x = j % N;
        out[j] = z[fft_pos<N>(y) * P + fft_pos<N>(x)].x * inv + m * (hw[y] * hw[x]);
    }
}

__global__ __launch_bounds__(NT) void k_mosaic(const BurstTable bt, const float *__restrict__ all_patches, int N,
                                               int stride, int window, const float *__restrict__ hann) {
    const int64_t gidx = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (gidx >= bt.pixels) return;
    const BurstDesc &bd = bt.b[burst_of(bt, gidx, [](const BurstDesc &d) { return d.pix0; })];
    const int H = bd.H, W = bd.W, ny = bd.ny, nx = bd.nx;
    const float *patches = all_patches + (size_t)bd.patch0 * N * N;
    float *out = bd.out;
    const int64_t idx = gidx - bd.pix0;
    const int y = (int)(idx / W), x = (int)(idx % W);
    float num = 0.f, dy = 0.f, dx = 0.f;
    const int ky0 = y >= N ? (y - N) / stride : 0;
    const int kx0 = x >= N ? (x - N) / stride : 0;
    for (int kx = kx0; kx < nx; ++kx) {
        const int ox = min(kx * stride, W - N);
        if (ox > x) break;
        if (x < ox + N) dx += window ? hann[x - ox] : 1.0f;
    }
    for (int ky = ky0; ky < ny; ++ky) {
        const int oy = min(ky * stride, H - N);
        if (oy > y) break;
        if (y >= oy + N) continue;
        dy += window ? hann[y - oy] : 1.0f;
        for (int kx = kx0; kx < nx; ++kx) {
            const int ox = min(kx * stride, W - N);
            if (ox > x) break;
            if (x >= ox + N) continue;
            num += patches[((size_t)(ky * nx + kx) * N + (y - oy)) * N + (x - ox)];
        }
    }
    const float den = dy * dx;
    out[idx] = den >= 1e-3f ? num / den : 0.f;
}

template <int N>
hipError_t launch_synth_t(const SynthArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(k_synth<N>, dim3(a.bt.patches), dim3(NT), 0, st, a.nW, a.Wxy, a.amp, a.phasor, a.filt,
                       a.mu, a.window, a.hann, a.twiddle, a.patch_buf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !a.mosaic || a.bt.pixels == 0) return e;
    hipLaunchKernelGGL(k_mosaic, dim3((unsigned)((a.bt.pixels + NT - 1) / NT)), dim3(NT), 0, st, a.bt, a.patch_buf,
                       N, a.stride, a.window, a.hann);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_synth(const SynthArgs &a, hipStream_t st) {
    if (a.bt.patches == 0) return hipSuccess;
    return a.N == 128 ? launch_synth_t<128>(a, st) : launch_synth_t<64>(a, st);
}

}  // namespace nvsm
