// Device helpers shared by the gfx950 kernels: complex arithmetic, small
// in-register DFTs, and an in-place 2-D FFT of an N x N tile held in LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nvsm {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

// exp(-2 pi i k / 16), k = 0..7, the exact values rounded to float:
// cos(pi/8) = 0.92387953251128675613, sin(pi/8) = 0.38268343236508977173,
// cos(pi/4) = sin(pi/4) = 0.70710678118654752440.
__device__ __forceinline__ float2 tw16(int k) {
    switch (k & 7) {
        case 0: return make_float2(1.0f, 0.0f);
        case 1: return make_float2(0.92387953251128675613f, -0.38268343236508977173f);
        case 2: return make_float2(0.70710678118654752440f, -0.70710678118654752440f);
        case 3: return make_float2(0.38268343236508977173f, -0.92387953251128675613f);
        case 4: return make_float2(0.0f, -1.0f);
        case 5: return make_float2(-0.38268343236508977173f, -0.92387953251128675613f);
        case 6: return make_float2(-0.70710678118654752440f, -0.70710678118654752440f);
        default: return make_float2(-0.92387953251128675613f, -0.38268343236508977173f);
    }
}

// d * exp(-2 pi i k / 16) with the trivial factors done exactly.
template <int K>
__device__ __forceinline__ float2 rot16(float2 d) {
    if constexpr ((K & 7) == 0) return d;
    else if constexpr ((K & 7) == 4) return make_float2(d.y, -d.x);
    else return cmul(d, tw16(K));
}

template <int L> struct Log2;
template <> struct Log2<2> { static constexpr int v = 1; };
template <> struct Log2<4> { static constexpr int v = 2; };
template <> struct Log2<8> { static constexpr int v = 3; };
template <> struct Log2<16> { static constexpr int v = 4; };

template <int L>
__host__ __device__ constexpr int bitrev(int i) {
    int r = 0;
    for (int b = 0; b < Log2<L>::v; ++b) r |= ((i >> b) & 1) << (Log2<L>::v - 1 - b);
    return r;
}

// One radix-2 decimation-in-frequency stage of span S on x[0..L).
template <int L, int S, int J = 0, int B = 0>
__device__ __forceinline__ void dif_stage(float2 *x) {
    if constexpr (B < L) {
        if constexpr (J < S) {
            float2 a = x[B + J], b = x[B + J + S];
            x[B + J] = cadd(a, b);
            x[B + J + S] = rot16<J * (8 / S)>(csub(a, b));
            dif_stage<L, S, J + 1, B>(x);
        } else {
            dif_stage<L, S, 0, B + 2 * S>(x);
        }
    }
}

template <int L, int S>
__device__ __forceinline__ void dif_all(float2 *x) {
    if constexpr (S >= 1) {
        dif_stage<L, S>(x);
        dif_all<L, S / 2>(x);
    }
}

// In-register DFT of length L (8 or 16), forward sign.  On return x[i]
// holds X[bitrev(i)].
template <int L>
__device__ __forceinline__ void dft_inreg(float2 *x) { dif_all<L, L / 2>(x); }

// Geometry of the in-LDS N-point transform: N = R1 * R2.
template <int N> struct FftGeom;
template <> struct FftGeom<64> { static constexpr int R1 = 8, R2 = 8; };
template <> struct FftGeom<128> { static constexpr int R1 = 8, R2 = 16; };

// Storage position of frequency k after fft2d_lds (per axis).
template <int N>
__host__ __device__ constexpr int fft_pos(int k) {
    return FftGeom<N>::R1 * (k % FftGeom<N>::R2) + k / FftGeom<N>::R2;
}

template <int N> struct LdsPitch { static constexpr int v = N + 1; };

// Stored spectrum of one (patch, frame): rows uy = -SPEC_NEG_ROWS .. N/2-1
// of I(ux, uy), row-major, ux in DFT order (column ux mod N).  The rows
// below 0 are the conjugate mirrors I(ux, -uy) = conj I(-ux, uy), kept so
// that every value the bispectrum needs is a plain load.
constexpr int SPEC_NEG_ROWS = 16;
template <int N> struct SpecRows {
    static constexpr int ROWS = N / 2 + SPEC_NEG_ROWS;
    static constexpr int FS = ROWS * N;
};

// In-place forward 2-D DFT (unnormalised, exp(-2 pi i ...)) of the N x N
// complex tile z[y * PITCH + x] in LDS, by NT threads.  tw[k] =
// exp(-2 pi i k / N).  Input in natural order; on return frequency
// (ky, kx) sits at z[fft_pos(ky) * PITCH + fft_pos(kx)].  Each axis is a
// radix-R2 pass over stride-R1 subsequences with twiddles, then a radix-R1
// pass over contiguous groups.  Ends with a barrier.
template <int N, int NT>
__device__ __forceinline__ void fft2d_lds_inline(float2 *z, const float2 *tw) {
    constexpr int R1 = FftGeom<N>::R1, R2 = FftGeom<N>::R2, P = LdsPitch<N>::v;
    const int tid = threadIdx.x;
    // axis 0 = along x (rows), axis 1 = along y (columns)
#pragma unroll
    for (int axis = 0; axis < 2; ++axis) {
        const int es = axis == 0 ? 1 : P;   // element step along the axis
        const int ls = axis == 0 ? P : 1;   // step between lines
        // pass A: for each line and n1, DFT over n2 of x[n1 + R1 n2]
#pragma unroll 2
        for (int t = tid; t < N * R1; t += NT) {
            const int line = t % N, n1 = t / N;
            float2 v[R2];
            float2 *base = z + line * ls + n1 * es;
#pragma unroll
            for (int n2 = 0; n2 < R2; ++n2) v[n2] = base[n2 * R1 * es];
            dft_inreg<R2>(v);
#pragma unroll
            for (int i = 0; i < R2; ++i) {
                const int k2 = bitrev<R2>(i);
                base[k2 * R1 * es] = cmul(v[i], tw[(n1 * k2) % N]);
            }
        }
        __syncthreads();
        // pass B: for each line and k2, DFT over n1 of the contiguous group
#pragma unroll 2
        for (int t = tid; t < N * R2; t += NT) {
            const int line = t % N, k2 = t / N;
            float2 v[R1];
            float2 *base = z + line * ls + (R1 * k2) * es;
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) v[n1] = base[n1 * es];
            dft_inreg<R1>(v);
#pragma unroll
            for (int i = 0; i < R1; ++i) base[bitrev<R1>(i) * es] = v[i];
        }
        __syncthreads();
    }
}
// The same, left to the compiler to inline or call (a call keeps the
// transform's registers out of a caller that holds many of its own).
template <int N, int NT>
__device__ void fft2d_lds(float2 *z, const float2 *tw) {
    fft2d_lds_inline<N, NT>(z, tw);
}

// A wave-uniform pointer held in scalar registers, opaque to the optimizer:
// loads at (base + 32-bit lane offset) then use scalar-base addressing
// instead of per-lane 64-bit address arithmetic.
typedef const __attribute__((address_space(1))) char *gptr_c;
__device__ __forceinline__ gptr_c uniform_ptr(const void *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (gptr_c)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float2 load_global_f2(gptr_c base, unsigned byte_off) {
    const unsigned long long v = *(const __attribute__((address_space(1))) unsigned long long *)(base + byte_off);
    return make_float2(__uint_as_float((unsigned)v), __uint_as_float((unsigned)(v >> 32)));
}
// The same for stores.
typedef __attribute__((address_space(1))) char *gptr_m;
__device__ __forceinline__ gptr_m uniform_ptr_m(void *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (gptr_m)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ void store_global_f2(gptr_m base, unsigned byte_off, float2 v) {
    *(__attribute__((address_space(1))) unsigned long long *)(base + byte_off) =
        (unsigned long long)__float_as_uint(v.x) | ((unsigned long long)__float_as_uint(v.y) << 32);
}

// Workgroup id remapped so that consecutive logical ids stay on one XCD:
// hardware dispatches workgroup b to XCD b % 8.
__device__ __forceinline__ int xcd_remap(int b, int total) {
    const int x = b & 7, n = b >> 3, q = total >> 3, r = total & 7;
    return x * q + (x < r ? x : r) + n;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Kahan step: (s, c) += x.
__device__ __forceinline__ void kahan_add(float &s, float &c, float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

}  // namespace nvsm
