// Ingest: subimage cut, taper, 2-D FFT and the power/mean accumulation of
// the Eq. 1 numerator.  One workgroup per (patch, group of frames), over
// all patches of the bursts of the launch.
//
// Two real frames a, b are transformed together as z = qa + i qb; with
// Z = FFT2(z), Ia(u) = (Z(u) + conj Z(-u)) / 2 and
// Ib(u) = (Z(u) - conj Z(-u)) / (2i).
#include "device_common.hpp"
#include "kernels.hpp"

#include <algorithm>

namespace nvsm {

namespace {

constexpr int NT = 256;
// The transform kernels hold one workgroup per CU (the tile fills most of
// LDS), so they run 8 waves to hide latency.
constexpr int FT = 512;

// Four consecutive pixels of a row, loaded as one vector when the layout
// allows it (VEC), else one by one.
template <typename T, bool VEC> struct Quad;
template <> struct Quad<uint16_t, true> {
    ushort4 v;
    __device__ void load(const uint16_t *p) { v = *(const ushort4 *)p; }
    __device__ void load(gptr_c base, unsigned off) {
        const unsigned long long u = *(const __attribute__((address_space(1))) unsigned long long *)(base + off);
        v = make_ushort4((unsigned short)u, (unsigned short)(u >> 16), (unsigned short)(u >> 32),
                         (unsigned short)(u >> 48));
    }
    __device__ float operator[](int i) const { return (float)(i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w); }
};
template <> struct Quad<float, true> {
    float4 v;
    __device__ void load(const float *p) { v = *(const float4 *)p; }
    __device__ void load(gptr_c base, unsigned off) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 u = *(const __attribute__((address_space(1))) f4 *)(base + off);
        v = make_float4(u.x, u.y, u.z, u.w);
    }
    __device__ float operator[](int i) const { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }
};
template <typename T> struct Quad<T, false> {
    float e[4];
    __device__ void load(const T *p) {
#pragma unroll
        for (int i = 0; i < 4; ++i) e[i] = (float)p[i];
    }
    __device__ void load(gptr_c base, unsigned off) {
        const __attribute__((address_space(1))) T *p = (const __attribute__((address_space(1))) T *)(base + off);
#pragma unroll
        for (int i = 0; i < 4; ++i) e[i] = (float)p[i];
    }
    __device__ float operator[](int i) const { return e[i]; }
};

// Storage position of frequency k after the transform (as fft_pos), in
// unsigned arithmetic for indices the optimizer cannot bound.
template <int N>
__device__ __forceinline__ unsigned fft_pos_u(unsigned k) {
    return FftGeom<N>::R1 * (k % FftGeom<N>::R2) + k / FftGeom<N>::R2;
}

// Threads of an ingest workgroup: 8 waves (2 per SIMD), whose registers
// hold the next frame pair's pixels through the transform (16 waves at 128
// registers per lane could not).  The transform is inlined into the kernel
// (as a call it kept registers of its own and waited for every load in
// flight at its entry).
template <typename T> constexpr int ingest_threads() { return 512; }

template <int N, typename T, bool VEC>
__global__ __launch_bounds__(ingest_threads<T>()) void k_ingest(const BurstTable bt, int stride, int chunk_frames, int window,
                                               float inv_wsum, const float2 *__restrict__ twiddle,
                                               const float *__restrict__ hann,
                                               float2 *__restrict__ spectra, float *__restrict__ ppart,
                                               float *__restrict__ mpart, float *__restrict__ mupart) {
    constexpr int IT = ingest_threads<T>();
    constexpr int P = LdsPitch<N>::v;
    constexpr int HALF = N / 2;
    constexpr int NP = (HALF + 1) * N;           // power rows 0..N/2
    constexpr int NPT = (NP + IT - 1) / IT;
    constexpr int QPT = N * N / 4 / IT;          // pixel quads per thread and frame
    __shared__ float2 z[N * P];
    __shared__ float2 tw[N];
    __shared__ float hw[N];
    __shared__ float red[2][IT / 64];

    const int L = xcd_remap(blockIdx.x, bt.ingest_wgs);
    const int b = burst_of(bt, L, [](const BurstDesc &d) { return (int64_t)d.ingest0; });
    const BurstDesc &bd = bt.b[b];
    const int F = bd.F, H = bd.H, W = bd.W, nx = bd.nx;
    const int64_t pitch = bd.pitch;
    const T *frames = (const T *)bd.frames;
    const int nchunks = (F + chunk_frames - 1) / chunk_frames;
    const int local = L - bd.ingest0;
    const int lpatch = local / nchunks, chunk = local % nchunks;
    const int py = lpatch / nx, px = lpatch % nx;
    const int y0 = min(py * stride, H - N), x0 = min(px * stride, W - N);
    const int f0 = chunk * chunk_frames, f1 = min(F, f0 + chunk_frames);
    const int tid = threadIdx.x;
    for (int i = tid; i < N; i += IT) {
        tw[i] = twiddle[i];
        hw[i] = window ? hann[i] : 1.0f;
    }
    // power sums of this frame group: plain FP32 over the group (at most
    // CHUNK_FRAMES frames); the groups are combined with Kahan sums later
    float ps[NPT];
#pragma unroll
    for (int i = 0; i < NPT; ++i) ps[i] = 0.f;
    float m10s[2] = {0.f, 0.f}, m10c[2] = {0.f, 0.f}, m01s[2] = {0.f, 0.f}, m01c[2] = {0.f, 0.f};
    float mus = 0.f, muc = 0.f;
    constexpr int FS = SpecRows<N>::FS;          // float2 per stored frame spectrum
    const size_t spec_patch = (size_t)(bd.spec0 + (int64_t)lpatch * F) * FS;

    // raw pixels of the current frame pair (wave-uniform frame bases, 32-bit
    // lane offsets).  The next pair's are requested after the transform,
    // before the record stores (see below).
    Quad<T, VEC> qa[QPT], qb[QPT];
    auto load_pair = [&](int fa) __attribute__((always_inline)) {
        const int fb = min(fa + 1, f1 - 1);
        const gptr_c pa = uniform_ptr(frames + (size_t)fa * H * pitch + (size_t)y0 * pitch + x0);
        const gptr_c pb = uniform_ptr(frames + (size_t)fb * H * pitch + (size_t)y0 * pitch + x0);
        // the thread index, opaque to the optimizer: the offsets are formed
        // here rather than kept (spilled) across the loop.  Quad j of a
        // thread lies 4 IT / N rows below its quad 0, in the same columns, so
        // one per-lane offset and a uniform step give them all (unsigned:
        // the offsets are 32-bit by the host's checks).
        unsigned tid_l;
        asm volatile("v_mov_b32 %0, %1" : "=v"(tid_l) : "v"(tid));
        static_assert(4 * IT % N == 0, "whole rows between the quads of a thread");
        const unsigned off0 = ((4u * tid_l) / N * (unsigned)pitch + (4u * tid_l) % N) * (unsigned)sizeof(T);
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            const unsigned off = off0 + (unsigned)(j * (4 * IT / N)) * (unsigned)pitch * (unsigned)sizeof(T);
            qa[j].load(pa, off);
            qb[j].load(pb, off);
        }
    };
    __syncthreads();

    load_pair(f0);
    // all of the first pair here, so that at the loop's head only the loads
    // of a pass's prefetch are waited for (not the stores that follow them)
    __builtin_amdgcn_s_waitcnt(0x0f70);          // vmcnt(0)
    for (int fa = f0; fa < f1; fa += 2) {
        const int fb = fa + 1;
        const bool hasb = fb < f1;
        // weighted sums (compensated); the pixels stay in registers
        float sa = 0.f, ca = 0.f, sb = 0.f, cb = 0.f;
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            const int q = j * IT + tid, y = (4 * q) / N, x = (4 * q) % N;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float va = qa[j][e], vb = hasb ? qb[j][e] : 0.f;
                const float w = hw[y] * hw[x + e];
                kahan_add(sa, ca, w * va);
                kahan_add(sb, cb, w * vb);
            }
        }
        float ra = wave_sum(sa - ca), rb = wave_sum(sb - cb);
        if ((tid & 63) == 0) { red[0][tid >> 6] = ra; red[1][tid >> 6] = rb; }
        __syncthreads();
        float mua = 0.f, mub = 0.f;
#pragma unroll
        for (int k = 0; k < IT / 64; ++k) { mua += red[0][k]; mub += red[1][k]; }
        mua *= inv_wsum;
        mub *= inv_wsum;
        if (tid == 0) {
            kahan_add(mus, muc, mua);
            if (hasb) kahan_add(mus, muc, mub);
        }
        // the mean-removed, tapered pixels to LDS (the previous pair's
        // transform was read before the loop's last barrier)
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            const int q = j * IT + tid, y = (4 * q) / N, x = (4 * q) % N;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float w = hw[y] * hw[x + e];
                const float va = qa[j][e], vb = hasb ? qb[j][e] : 0.f;
                z[y * P + x + e] = make_float2((va - mua) * w, hasb ? (vb - mub) * w : 0.f);
            }
        }
        __syncthreads();
        // the next pair's pixels, requested now (into the registers this
        // pair's pixels left), so that they arrive during the transform, and
        // before this pair's record stores: loads and stores share one
        // counter, so the next pair then waits for its pixels only.  Every
        // pass issues the same loads and stores (past the group's end the
        // last frame is loaded again, unused; a missing second frame's stores
        // go to the first frame's record, ahead of the first frame's own), so
        // the compiler knows how many are in flight.
        load_pair(min(fa + 2, f1 - 1));
        fft2d_lds_inline<N, IT>(z, tw);
        // records of the two frames: wave-uniform bases, 32-bit lane offsets
        const gptr_m rec_a = uniform_ptr_m(spectra + spec_patch + (size_t)fa * FS);
        const gptr_m rec_b = uniform_ptr_m(spectra + spec_patch + (size_t)(hasb ? fb : fa) * FS);
        unsigned tid_o;              // opaque thread index (addresses formed here, unsigned)
        asm volatile("v_mov_b32 %0, %1" : "=v"(tid_o) : "v"(tid));
        // I_a and I_b of frequency (ux, uy) from the transform of z = a + i b
        auto split = [&](unsigned ux, unsigned uy, float2 &Ia, float2 &Ib) __attribute__((always_inline)) {
            const float2 Z = z[fft_pos_u<N>(uy) * P + fft_pos_u<N>(ux)];
            const float2 Zm = z[fft_pos_u<N>((N - uy) & (N - 1)) * P + fft_pos_u<N>((N - ux) & (N - 1))];
            Ia = make_float2(0.5f * (Z.x + Zm.x), 0.5f * (Z.y - Zm.y));
            Ib = make_float2(0.5f * (Z.y + Zm.y), -0.5f * (Z.x - Zm.x));
        };
        // rows 0..N/2-1: the record rows and the power; row N/2: the power
        static_assert(HALF * N % IT == 0 && SPEC_NEG_ROWS * N % IT == 0, "whole rows per pass");
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const unsigned j = k * IT + tid_o;
            if (k * IT + tid < NP) {
                const unsigned uy = j / N, ux = j % N;
                float2 Ia, Ib;
                split(ux, uy, Ia, Ib);
                ps[k] += Ia.x * Ia.x + Ia.y * Ia.y;
                if (hasb) ps[k] += Ib.x * Ib.x + Ib.y * Ib.y;
                if (k * IT < HALF * N) {
                    const unsigned o = ((uy + SPEC_NEG_ROWS) * N + ux) * (unsigned)sizeof(float2);
                    store_global_f2(rec_b, o, Ib);
                    store_global_f2(rec_a, o, Ia);
                }
                if (k * IT + tid == 1) {   // u = (1, 0)
                    kahan_add(m10s[0], m10c[0], Ia.x); kahan_add(m10s[1], m10c[1], Ia.y);
                    if (hasb) { kahan_add(m10s[0], m10c[0], Ib.x); kahan_add(m10s[1], m10c[1], Ib.y); }
                }
                if (k * IT + tid == N) {   // u = (0, 1)
                    kahan_add(m01s[0], m01c[0], Ia.x); kahan_add(m01s[1], m01c[1], Ia.y);
                    if (hasb) { kahan_add(m01s[0], m01c[0], Ib.x); kahan_add(m01s[1], m01c[1], Ib.y); }
                }
            }
        }
        // the conjugate mirrors I(-u) = conj I(u) of rows 1..16 in rows -1..-16
#pragma unroll
        for (int k = 0; k < SPEC_NEG_ROWS * N / IT; ++k) {
            const unsigned j = k * IT + tid_o;
            const unsigned uy = 1 + j / N, ux = j % N;
            float2 Ia, Ib;
            split(ux, uy, Ia, Ib);
            const unsigned om = ((SPEC_NEG_ROWS - uy) * N + ((N - ux) & (N - 1))) * (unsigned)sizeof(float2);
            store_global_f2(rec_b, om, conjf2(Ib));
            store_global_f2(rec_a, om, conjf2(Ia));
        }
        __syncthreads();
    }
    // partial sums of this frame group, at the workgroup's index
    float *pp = ppart + (size_t)L * NP;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int j = k * IT + tid;
        if (j < NP) pp[j] = ps[k];
    }
    float *mp = mpart + (size_t)L * 4;
    if (tid == 1 % IT) { mp[0] = m10s[0] - m10c[0]; mp[1] = m10s[1] - m10c[1]; }
    if (tid == N % IT) { mp[2] = m01s[0] - m01c[0]; mp[3] = m01s[1] - m01c[1]; }
    if (tid == 0) mupart[L] = mus - muc;
}

// Sums the frame groups (compensated) and divides by F; mirrors the power
// spectrum rows N/2+1..N-1 from P(-u) = P(u).
template <int N>
__global__ __launch_bounds__(NT) void k_acc_finalize(const BurstTable bt, int chunk_frames,
                                                     const float *__restrict__ ppart,
                                                     const float *__restrict__ mpart,
                                                     const float *__restrict__ mupart,
                                                     float *__restrict__ power, float *__restrict__ mean_spec,
                                                     float *__restrict__ mu) {
    constexpr int HALF = N / 2, NP = (HALF + 1) * N;
    const int patch = blockIdx.x;
    const int b = burst_of(bt, patch, [](const BurstDesc &d) { return (int64_t)d.patch0; });
    const BurstDesc &bd = bt.b[b];
    const int nchunks = (bd.F + chunk_frames - 1) / chunk_frames;
    const float invF = 1.0f / (float)bd.F;
    const size_t wg0 = (size_t)bd.ingest0 + (size_t)(patch - bd.patch0) * nchunks;   // its first ingest workgroup
    const float *pp = ppart + wg0 * NP;
    for (int j = threadIdx.x; j < N * N; j += NT) {
        const int uy = j / N, ux = j % N;
        const int src = uy <= HALF ? j : ((N - uy) * N + ((N - ux) & (N - 1)));
        float s = 0.f, c = 0.f;
        for (int k = 0; k < nchunks; ++k) kahan_add(s, c, pp[(size_t)k * NP + src]);
        power[(size_t)patch * N * N + j] = (s - c) * invF;
    }
    if (threadIdx.x < 4) {
        float s = 0.f, c = 0.f;
        for (int k = 0; k < nchunks; ++k) kahan_add(s, c, mpart[(wg0 + k) * 4 + threadIdx.x]);
        mean_spec[(size_t)patch * 4 + threadIdx.x] = (s - c) * invF;
    }
    if (threadIdx.x == 4) {
        float s = 0.f, c = 0.f;
        for (int k = 0; k < nchunks; ++k) kahan_add(s, c, mupart[wg0 + k]);
        mu[patch] = (s - c) * invF;
    }
}

// Streaming form of k_acc_finalize for one burst: adds the frame groups of
// this launch to running compensated sums kept between launches (from zero
// when first), sc = (sum, compensation) per value: power rows 0..N/2, the
// two mean spectrum values and the mean level.  last != 0: then writes the
// means over all frames, (sum - comp) * inv_total, as k_acc_finalize does.
template <int N>
__global__ __launch_bounds__(NT) void k_acc_stream(int nchunks, const float *__restrict__ ppart,
                                                   const float *__restrict__ mpart,
                                                   const float *__restrict__ mupart, float2 *__restrict__ psc,
                                                   float2 *__restrict__ msc, float2 *__restrict__ musc, int first,
                                                   int last,
                                                   float inv_total, float *__restrict__ power,
                                                   float *__restrict__ mean_spec, float *__restrict__ mu) {
    constexpr int HALF = N / 2, NP = (HALF + 1) * N;
    const int patch = blockIdx.x;
    const float *pp = ppart + (size_t)patch * nchunks * NP;
    float2 *ps = psc + (size_t)patch * NP;
    for (int j = threadIdx.x; j < NP; j += NT) {
        float2 v = first ? make_float2(0.f, 0.f) : ps[j];
        for (int k = 0; k < nchunks; ++k) kahan_add(v.x, v.y, pp[(size_t)k * NP + j]);
        ps[j] = v;
    }
    if (threadIdx.x < 4) {
        float2 v = first ? make_float2(0.f, 0.f) : msc[(size_t)patch * 4 + threadIdx.x];
        for (int k = 0; k < nchunks; ++k) kahan_add(v.x, v.y, mpart[((size_t)patch * nchunks + k) * 4 + threadIdx.x]);
        msc[(size_t)patch * 4 + threadIdx.x] = v;
        if (last) mean_spec[(size_t)patch * 4 + threadIdx.x] = (v.x - v.y) * inv_total;
    }
    if (threadIdx.x == 4) {
        float2 v = first ? make_float2(0.f, 0.f) : musc[patch];
        for (int k = 0; k < nchunks; ++k) kahan_add(v.x, v.y, mupart[(size_t)patch * nchunks + k]);
        musc[patch] = v;
        if (last) mu[patch] = (v.x - v.y) * inv_total;
    }
    if (!last) return;
    __syncthreads();
    for (int j = threadIdx.x; j < N * N; j += NT) {
        const int uy = j / N, ux = j % N;
        const int src = uy <= HALF ? j : ((N - uy) * N + ((N - ux) & (N - 1)));
        const float2 v = ps[src];
        power[(size_t)patch * N * N + j] = (v.x - v.y) * inv_total;
    }
}

template <int N, typename T>
hipError_t launch_ingest_t(const IngestArgs &a, hipStream_t st) {
    if (a.vec)
        hipLaunchKernelGGL((k_ingest<N, T, true>), dim3(a.bt.ingest_wgs), dim3(ingest_threads<T>()), 0, st, a.bt, a.stride,
                           a.chunk_frames, a.window, a.inv_wsum, a.twiddle, a.hann, a.spectra, a.ppart, a.mpart,
                           a.mupart);
    else
        hipLaunchKernelGGL((k_ingest<N, T, false>), dim3(a.bt.ingest_wgs), dim3(ingest_threads<T>()), 0, st, a.bt, a.stride,
                           a.chunk_frames, a.window, a.inv_wsum, a.twiddle, a.hann, a.spectra, a.ppart, a.mpart,
                           a.mupart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.stream_mode == 0) {
        hipLaunchKernelGGL((k_acc_finalize<N>), dim3(a.bt.patches), dim3(NT), 0, st, a.bt, a.chunk_frames,
                           a.ppart, a.mpart, a.mupart, a.power, a.mean_spec, a.mu);
    } else {
        const int nchunks = (a.bt.b[0].F + a.chunk_frames - 1) / a.chunk_frames;
        hipLaunchKernelGGL((k_acc_stream<N>), dim3(a.bt.patches), dim3(NT), 0, st, nchunks, a.ppart, a.mpart,
                           a.mupart, a.psc, a.msc, a.musc, a.stream_first, a.stream_mode == 2 ? 1 : 0, a.inv_total,
                           a.power,
                           a.mean_spec, a.mu);
    }
    return hipGetLastError();
}

// Photon-noise terms of one (patch, frame group), over the ingest grid.
// Each frame is transformed as z = (p - mu) t + i (p - mu) t^2: both halves
// have the scale of the fluctuations, so the FP32 rounding of one does not
// swamp the other.  One FFT gives I(u) = (Z(u) + conj Z(-u)) / 2 and
// Y(u) = (Z(u) - conj Z(-u)) / (2i), and Q(u) = (Y(u) + mu D(u)) / G with D
// the transform of t^2 (for the periodic Hann taper the product of
// 3N/8, -N/4, N/16 at per-axis frequency 0, +-1, +-2 and 0 elsewhere; N^2
// at u = 0 without taper).  The group's sums of conj I(u) Q(u) (rows
// 0..N/2), of q0 = sum(t^2 p) / G and of T = sum(t^3 p) / G^2 go to the
// workgroup's partials.
// DFT of the squared taper at (ux, uy) (indices mod N): real, separable.
template <int N>
__device__ __forceinline__ float taper2_dft(int window, int ux, int uy) {
    if (!window) return (ux == 0 && uy == 0) ? (float)(N * N) : 0.f;
    auto axis = [](int k) {
        const int m = k <= N / 2 ? k : k - N;          // signed frequency
        return m == 0 ? 0.375f * N : (m == 1 || m == -1) ? -0.25f * N : (m == 2 || m == -2) ? 0.0625f * N : 0.f;
    };
    return axis(ux) * axis(uy);
}

template <int N, typename T, bool VEC>
__global__ __launch_bounds__(FT) void k_noise(const BurstTable bt, int stride, int chunk_frames, int window,
                                              float inv_wsum, float inv_gain, const float2 *__restrict__ twiddle,
                                              const float *__restrict__ hann, float2 *__restrict__ cpart,
                                              float *__restrict__ spart) {
    constexpr int P = LdsPitch<N>::v;
    constexpr int HALF = N / 2;
    constexpr int NP = (HALF + 1) * N;
    constexpr int NPT = (NP + FT - 1) / FT;
    constexpr int QPT = N * N / 4 / FT;
    __shared__ float2 z[N * P];
    __shared__ float2 tw[N];
    __shared__ float hw[N];
    __shared__ float red[3][FT / 64];

    const int L = xcd_remap(blockIdx.x, bt.ingest_wgs);
    const int b = burst_of(bt, L, [](const BurstDesc &d) { return (int64_t)d.ingest0; });
    const BurstDesc &bd = bt.b[b];
    const int F = bd.F, H = bd.H, W = bd.W, nx = bd.nx;
    const int64_t pitch = bd.pitch;
    const T *frames = (const T *)bd.frames;
    const int nchunks = (F + chunk_frames - 1) / chunk_frames;
    const int local = L - bd.ingest0;
    const int lpatch = local / nchunks, chunk = local % nchunks;
    const int py = lpatch / nx, px = lpatch % nx;
    const int y0 = min(py * stride, H - N), x0 = min(px * stride, W - N);
    const int f0 = chunk * chunk_frames, f1 = min(F, f0 + chunk_frames);
    const int tid = threadIdx.x;
    for (int i = tid; i < N; i += FT) {
        tw[i] = twiddle[i];
        hw[i] = window ? hann[i] : 1.0f;
    }
    float2 cs[NPT];
#pragma unroll
    for (int i = 0; i < NPT; ++i) cs[i] = make_float2(0.f, 0.f);
    float q0s = 0.f, q0c = 0.f, ts = 0.f, tc = 0.f;
    // the pixels of a frame stay in registers until tapered; the next
    // frame's are requested once the tile is written, so that they arrive
    // during the transform (wave-uniform frame base, 32-bit lane offsets)
    Quad<T, VEC> v[QPT];
    auto load_frame = [&](int f) __attribute__((always_inline)) {
        const gptr_c pf = uniform_ptr(frames + (size_t)f * H * pitch + (size_t)y0 * pitch + x0);
        unsigned tid_l;                // opaque: the offsets are formed here, not kept
        asm volatile("v_mov_b32 %0, %1" : "=v"(tid_l) : "v"(tid));
        static_assert(4 * FT % N == 0, "whole rows between the quads of a thread");
        const unsigned off0 = ((4u * tid_l) / N * (unsigned)pitch + (4u * tid_l) % N) * (unsigned)sizeof(T);
#pragma unroll
        for (int j = 0; j < QPT; ++j)
            v[j].load(pf, off0 + (unsigned)(j * (4 * FT / N)) * (unsigned)pitch * (unsigned)sizeof(T));
    };
    __syncthreads();

    load_frame(f0);
    for (int f = f0; f < f1; ++f) {
        float s1 = 0.f, c1 = 0.f, s2 = 0.f, s3 = 0.f;
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            const int q = j * FT + tid, y = (4 * q) / N, x = (4 * q) % N;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float w = hw[y] * hw[x + e];
                const float wp = w * v[j][e];
                kahan_add(s1, c1, wp);
                s2 += w * wp;
                s3 += w * w * wp;
            }
        }
        const float r1 = wave_sum(s1 - c1), r2 = wave_sum(s2), r3 = wave_sum(s3);
        if ((tid & 63) == 0) { red[0][tid >> 6] = r1; red[1][tid >> 6] = r2; red[2][tid >> 6] = r3; }
        __syncthreads();
        float mu = 0.f, q0 = 0.f, t3 = 0.f;
#pragma unroll
        for (int k = 0; k < FT / 64; ++k) { mu += red[0][k]; q0 += red[1][k]; t3 += red[2][k]; }
        mu *= inv_wsum;
        if (tid == 0) {
            kahan_add(q0s, q0c, q0 * inv_gain);
            kahan_add(ts, tc, t3 * inv_gain * inv_gain);
        }
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            const int q = j * FT + tid, y = (4 * q) / N, x = (4 * q) % N;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float w = hw[y] * hw[x + e];
                const float d = (v[j][e] - mu) * w;
                z[y * P + x + e] = make_float2(d, d * w);
            }
        }
        __syncthreads();
        load_frame(min(f + 1, f1 - 1));   // (past the group's end: the last frame again, unused)
        fft2d_lds_inline<N, FT>(z, tw);
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int j = k * FT + tid;
            if (j < NP) {
                const int uy = j / N, ux = j % N;
                const float2 Z = z[fft_pos<N>(uy) * P + fft_pos<N>(ux)];
                const float2 Zm = z[fft_pos<N>((N - uy) & (N - 1)) * P + fft_pos<N>((N - ux) & (N - 1))];
                const float2 I = make_float2(0.5f * (Z.x + Zm.x), 0.5f * (Z.y - Zm.y));
                float2 Q = make_float2(0.5f * (Z.y + Zm.y), -0.5f * (Z.x - Zm.x));
                Q.x = (Q.x + mu * taper2_dft<N>(window, ux, uy)) * inv_gain;
                Q.y *= inv_gain;
                cs[k].x += I.x * Q.x + I.y * Q.y;         // conj(I) Q
                cs[k].y += I.x * Q.y - I.y * Q.x;
            }
        }
        __syncthreads();
    }
    float2 *cp = cpart + (size_t)L * NP;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int j = k * FT + tid;
        if (j < NP) cp[j] = cs[k];
    }
    if (tid == 0) {
        spart[(size_t)L * 2] = q0s - q0c;
        spart[(size_t)L * 2 + 1] = ts - tc;
    }
}

// Sums the frame groups of k_noise per patch (compensated), divides by F,
// writes C in the record layout of the spectra (rows -16 .. N/2-1, the rows
// below 0 as C(u) = conj C(-u)), and subtracts q0 from the patch's power
// spectrum.
template <int N>
__global__ __launch_bounds__(NT) void k_noise_finalize(const BurstTable bt, int chunk_frames,
                                                       const float2 *__restrict__ cpart,
                                                       const float *__restrict__ spart, float *__restrict__ power,
                                                       float2 *__restrict__ cgrid, float *__restrict__ nbar) {
    constexpr int HALF = N / 2, NP = (HALF + 1) * N;
    constexpr int FS = SpecRows<N>::FS;
    const int patch = blockIdx.x;
    const int b = burst_of(bt, patch, [](const BurstDesc &d) { return (int64_t)d.patch0; });
    const BurstDesc &bd = bt.b[b];
    const int nchunks = (bd.F + chunk_frames - 1) / chunk_frames;
    const float invF = 1.0f / (float)bd.F;
    const size_t wg0 = (size_t)bd.ingest0 + (size_t)(patch - bd.patch0) * nchunks;
    // every thread forms the same two means in the same order
    float q0 = 0.f, q0c = 0.f, t3 = 0.f, t3c = 0.f;
    for (int k = 0; k < nchunks; ++k) {
        kahan_add(q0, q0c, spart[(wg0 + k) * 2]);
        kahan_add(t3, t3c, spart[(wg0 + k) * 2 + 1]);
    }
    q0 = (q0 - q0c) * invF;
    t3 = (t3 - t3c) * invF;
    if (threadIdx.x == 0) {
        nbar[(size_t)patch * 2] = q0;
        nbar[(size_t)patch * 2 + 1] = t3;
    }
    const float2 *cp = cpart + wg0 * NP;
    for (int i = threadIdx.x; i < FS; i += NT) {
        const int y = i / N - SPEC_NEG_ROWS, x = i % N;
        const bool mirror = y < 0;
        const int j = mirror ? (-y) * N + ((N - x) & (N - 1)) : y * N + x;
        float sx = 0.f, cx = 0.f, sy = 0.f, cy = 0.f;
        for (int k = 0; k < nchunks; ++k) {
            const float2 v = cp[(size_t)k * NP + j];
            kahan_add(sx, cx, v.x);
            kahan_add(sy, cy, v.y);
        }
        const float im = (sy - cy) * invF;
        cgrid[(size_t)patch * FS + i] = make_float2((sx - cx) * invF, mirror ? -im : im);
    }
    float *pw = power + (size_t)patch * N * N;
    for (int j = threadIdx.x; j < N * N; j += NT) pw[j] -= q0;
}

// The streaming form of k_noise_finalize: one workgroup per patch adds the
// group's sums (its frame chunks in order, compensated) to the running
// pairs; the last group writes the means as k_noise_finalize does.  With
// one group holding every frame the means are those of k_noise_finalize bit
// for bit.
template <int N>
__global__ __launch_bounds__(NT) void k_noise_stream(const BurstTable bt, int chunk_frames,
                                                     const float2 *__restrict__ cpart,
                                                     const float *__restrict__ spart, int mode, int first,
                                                     float inv_total, float4 *__restrict__ csc,
                                                     float *__restrict__ ssc, float *__restrict__ power,
                                                     float2 *__restrict__ cgrid, float *__restrict__ nbar) {
    constexpr int HALF = N / 2, NP = (HALF + 1) * N;
    constexpr int FS = SpecRows<N>::FS;
    const int patch = blockIdx.x;
    const BurstDesc &bd = bt.b[0];
    const int nchunks = (bd.F + chunk_frames - 1) / chunk_frames;
    const size_t wg0 = (size_t)bd.ingest0 + (size_t)patch * nchunks;
    // every thread forms the same two sums in the same order
    float q0 = 0.f, q0c = 0.f, t3 = 0.f, t3c = 0.f;
    float *sp = ssc + (size_t)patch * 4;
    if (!first) {
        q0 = sp[0]; t3 = sp[1]; q0c = sp[2]; t3c = sp[3];
    }
    for (int k = 0; k < nchunks; ++k) {
        kahan_add(q0, q0c, spart[(wg0 + k) * 2]);
        kahan_add(t3, t3c, spart[(wg0 + k) * 2 + 1]);
    }
    __syncthreads();                              // every thread has read the running pair
    if (mode == 1) {
        if (threadIdx.x == 0) {
            sp[0] = q0; sp[1] = t3; sp[2] = q0c; sp[3] = t3c;
        }
    } else {
        q0 = (q0 - q0c) * inv_total;
        t3 = (t3 - t3c) * inv_total;
        if (threadIdx.x == 0) {
            nbar[(size_t)patch * 2] = q0;
            nbar[(size_t)patch * 2 + 1] = t3;
        }
    }
    const float2 *cp = cpart + wg0 * NP;
    float4 *cs = csc + (size_t)patch * NP;
    float2 *cg = cgrid + (size_t)patch * FS;
    for (int j = threadIdx.x; j < NP; j += NT) {
        float sx = 0.f, cx = 0.f, sy = 0.f, cy = 0.f;
        if (!first) {
            const float4 r = cs[j];
            sx = r.x; sy = r.y; cx = r.z; cy = r.w;
        }
        for (int k = 0; k < nchunks; ++k) {
            const float2 v = cp[(size_t)k * NP + j];
            kahan_add(sx, cx, v.x);
            kahan_add(sy, cy, v.y);
        }
        if (mode == 1) {
            cs[j] = make_float4(sx, sy, cx, cy);
            continue;
        }
        // means at their record place (rows 0 .. N/2 - 1), and the conjugate
        // mirrors of rows 1 .. SPEC_NEG_ROWS in rows -1 .. -SPEC_NEG_ROWS
        const int y = j / N, x = j % N;
        const float mx = (sx - cx) * inv_total, my = (sy - cy) * inv_total;
        if (y < HALF) cg[(y + SPEC_NEG_ROWS) * N + x] = make_float2(mx, my);
        if (y >= 1 && y <= SPEC_NEG_ROWS) cg[(SPEC_NEG_ROWS - y) * N + ((N - x) & (N - 1))] = make_float2(mx, -my);
    }
    if (mode == 2) {
        float *pw = power + (size_t)patch * N * N;
        for (int j = threadIdx.x; j < N * N; j += NT) pw[j] -= q0;
    }
}

template <int N, typename T>
hipError_t launch_noise_t(const NoiseArgs &na, hipStream_t st) {
    const IngestArgs &a = na.in;
    if (a.vec)
        hipLaunchKernelGGL((k_noise<N, T, true>), dim3(a.bt.ingest_wgs), dim3(FT), 0, st, a.bt, a.stride,
                           a.chunk_frames, a.window, a.inv_wsum, na.inv_gain, a.twiddle, a.hann, na.cpart,
                           na.spart);
    else
        hipLaunchKernelGGL((k_noise<N, T, false>), dim3(a.bt.ingest_wgs), dim3(FT), 0, st, a.bt, a.stride,
                           a.chunk_frames, a.window, a.inv_wsum, na.inv_gain, a.twiddle, a.hann, na.cpart,
                           na.spart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.stream_mode == 0)
        hipLaunchKernelGGL((k_noise_finalize<N>), dim3(a.bt.patches), dim3(NT), 0, st, a.bt, a.chunk_frames, na.cpart,
                           na.spart, a.power, na.cgrid, na.nbar);
    else
        hipLaunchKernelGGL((k_noise_stream<N>), dim3(a.bt.patches), dim3(NT), 0, st, a.bt, a.chunk_frames, na.cpart,
                           na.spart, a.stream_mode, a.stream_first, a.inv_total, na.csc, na.ssc, a.power, na.cgrid,
                           na.nbar);
    return hipGetLastError();
}

// Spectral-ratio sums of the seeing cubes: one workgroup per (cube, frame
// group); cube c is the N x N tile at (c / nx, c % nx) * N of frames
// [F][H][pitch].  Two frames per transform as in k_ingest (same taper and
// weighted-mean removal).  Only the box 0 <= uy <= B, |ux| <= B is kept:
// per entry e = uy (2B + 1) + ux + B the group's sums of I (re, im) and of
// |I|^2 go to part[L][e][0..2].
template <int N, typename T, bool VEC>
__global__ __launch_bounds__(FT) void k_ratio(const RatioArgs a) {
    constexpr int P = LdsPitch<N>::v;
    constexpr int QPT = N * N / 4 / FT;
    constexpr int MAXE = (RATIO_MAX_BINS + 3) * (2 * RATIO_MAX_BINS + 5);
    constexpr int EPT = (MAXE + FT - 1) / FT;
    __shared__ float2 z[N * P];
    __shared__ float2 tw[N];
    __shared__ float hw[N];
    __shared__ float red[2][FT / 64];
    const T *frames = (const T *)a.frames;
    const int64_t pitch = a.pitch;
    const int nchunks = (a.F + a.chunk_frames - 1) / a.chunk_frames;
    const int L = blockIdx.x;
    const int cube = L / nchunks, chunk = L % nchunks;
    const int y0 = (cube / a.nx) * N, x0 = (cube % a.nx) * N;
    const int f0 = chunk * a.chunk_frames, f1 = min(a.F, f0 + a.chunk_frames);
    const int B = a.B, bw = 2 * B + 1, nbox = (B + 1) * bw;
    const int tid = threadIdx.x;
    for (int i = tid; i < N; i += FT) {
        tw[i] = a.twiddle[i];
        hw[i] = a.window ? a.hann[i] : 1.0f;
    }
    float sm[EPT][3];
#pragma unroll
    for (int k = 0; k < EPT; ++k) sm[k][0] = sm[k][1] = sm[k][2] = 0.f;
    // the pixels of a frame pair (a lone last frame: loaded twice, the copy
    // unused); the next pair's are requested once the tile is written, so
    // that they arrive during the transform, as in k_ingest
    Quad<T, VEC> qa[QPT], qb[QPT];
    auto load_pair = [&](int fa) __attribute__((always_inline)) {
        const int fb = min(fa + 1, f1 - 1);
        const gptr_c pa = uniform_ptr(frames + (size_t)fa * a.H * pitch + (size_t)y0 * pitch + x0);
        const gptr_c pb = uniform_ptr(frames + (size_t)fb * a.H * pitch + (size_t)y0 * pitch + x0);
        unsigned tid_l;                // opaque: the offsets are formed here, not kept
        asm volatile("v_mov_b32 %0, %1" : "=v"(tid_l) : "v"(tid));
        static_assert(4 * FT % N == 0, "whole rows between the quads of a thread");
        const unsigned off0 = ((4u * tid_l) / N * (unsigned)pitch + (4u * tid_l) % N) * (unsigned)sizeof(T);
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            const unsigned off = off0 + (unsigned)(j * (4 * FT / N)) * (unsigned)pitch * (unsigned)sizeof(T);
            qa[j].load(pa, off);
            qb[j].load(pb, off);
        }
    };
    __syncthreads();
    load_pair(f0);
    for (int fa = f0; fa < f1; fa += 2) {
        const bool hasb = fa + 1 < f1;
        float sa = 0.f, ca = 0.f, sb = 0.f, cb = 0.f;
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            const int q = j * FT + tid, y = (4 * q) / N, x = (4 * q) % N;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float va = qa[j][e], vb = hasb ? qb[j][e] : 0.f;
                const float w = hw[y] * hw[x + e];
                kahan_add(sa, ca, w * va);
                kahan_add(sb, cb, w * vb);
            }
        }
        const float r0 = wave_sum(sa - ca), r1 = wave_sum(sb - cb);
        if ((tid & 63) == 0) { red[0][tid >> 6] = r0; red[1][tid >> 6] = r1; }
        __syncthreads();
        float mua = 0.f, mub = 0.f;
#pragma unroll
        for (int k = 0; k < FT / 64; ++k) { mua += red[0][k]; mub += red[1][k]; }
        mua *= a.inv_wsum;
        mub *= a.inv_wsum;
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            const int q = j * FT + tid, y = (4 * q) / N, x = (4 * q) % N;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float w = hw[y] * hw[x + e];
                const float va = qa[j][e], vb = hasb ? qb[j][e] : 0.f;
                z[y * P + x + e] = make_float2((va - mua) * w, hasb ? (vb - mub) * w : 0.f);
            }
        }
        __syncthreads();
        load_pair(min(fa + 2, f1 - 1));
        fft2d_lds_inline<N, FT>(z, tw);
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int e = k * FT + tid;
            if (e < nbox) {
                const int uy = e / bw, ux = (e % bw - B) & (N - 1);
                const float2 Z = z[fft_pos<N>(uy) * P + fft_pos<N>(ux)];
                const float2 Zm = z[fft_pos<N>((N - uy) & (N - 1)) * P + fft_pos<N>((N - ux) & (N - 1))];
                const float2 Ia = make_float2(0.5f * (Z.x + Zm.x), 0.5f * (Z.y - Zm.y));
                const float2 Ib = make_float2(0.5f * (Z.y + Zm.y), -0.5f * (Z.x - Zm.x));
                sm[k][0] += Ia.x;
                sm[k][1] += Ia.y;
                sm[k][2] += Ia.x * Ia.x + Ia.y * Ia.y;
                if (hasb) {
                    sm[k][0] += Ib.x;
                    sm[k][1] += Ib.y;
                    sm[k][2] += Ib.x * Ib.x + Ib.y * Ib.y;
                }
            }
        }
        __syncthreads();
    }
    float *pp = a.part + (size_t)L * nbox * 3;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int e = k * FT + tid;
        if (e < nbox) {
            pp[3 * e] = sm[k][0];
            pp[3 * e + 1] = sm[k][1];
            pp[3 * e + 2] = sm[k][2];
        }
    }
}

template <int N, typename T>
hipError_t launch_ratio_t(const RatioArgs &a, hipStream_t st) {
    const int nchunks = (a.F + a.chunk_frames - 1) / a.chunk_frames;
    const int grid = a.cubes * nchunks;
    if (a.vec)
        hipLaunchKernelGGL((k_ratio<N, T, true>), dim3(grid), dim3(FT), 0, st, a);
    else
        hipLaunchKernelGGL((k_ratio<N, T, false>), dim3(grid), dim3(FT), 0, st, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(NT) void k_zero(float4 *__restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

}  // namespace

hipError_t launch_zero(void *p, size_t bytes, hipStream_t st) {
    const int64_t n = (int64_t)(bytes / 16);
    if (n == 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((n + NT - 1) / NT, 8192);
    hipLaunchKernelGGL(k_zero, dim3(grid), dim3(NT), 0, st, (float4 *)p, n);
    return hipGetLastError();
}

hipError_t launch_noise(const NoiseArgs &na, hipStream_t st) {
    const IngestArgs &a = na.in;
    if (a.bt.patches == 0) return hipSuccess;
    if (a.N == 128) return a.f32 ? launch_noise_t<128, float>(na, st) : launch_noise_t<128, uint16_t>(na, st);
    return a.f32 ? launch_noise_t<64, float>(na, st) : launch_noise_t<64, uint16_t>(na, st);
}

hipError_t launch_ratio(const RatioArgs &a, hipStream_t st) {
    if (a.cubes < 1 || a.F < 2 || a.B < 3 || a.B > RATIO_MAX_BINS + 2 || a.chunk_frames < 1) return hipErrorInvalidValue;
    if (a.N == 128) return a.f32 ? launch_ratio_t<128, float>(a, st) : launch_ratio_t<128, uint16_t>(a, st);
    return a.f32 ? launch_ratio_t<64, float>(a, st) : launch_ratio_t<64, uint16_t>(a, st);
}

hipError_t launch_ingest(const IngestArgs &a, hipStream_t st) {
    if (a.bt.patches == 0) return hipSuccess;
    if (a.N == 128) return a.f32 ? launch_ingest_t<128, float>(a, st) : launch_ingest_t<128, uint16_t>(a, st);
    return a.f32 ? launch_ingest_t<64, float>(a, st) : launch_ingest_t<64, uint16_t>(a, st);
}

}  // namespace nvsm
