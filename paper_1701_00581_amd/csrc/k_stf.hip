// Model speckle transfer function by Monte Carlo: <|OTF|^2> (and <OTF>) over
// Kolmogorov phase screens across a circular pupil of diameter N/2 px in the
// N x N patch grid (the PSF is then Nyquist sampled on the patch grid).
//
// Screens: phase spectrum 0.023 r0^(-5/3) f^(-11/3) on the DFT frequencies
// (FFT method; a screen pair is the real and imaginary part of one complex
// transform) plus three subharmonic levels (Lane, Glindemann and Dainty
// 1992).  Random numbers: Philox4x32-10 (Salmon et al. 2011), key = the
// seed's two halves, counter (pair j, word w, stream m, 0); each word gives
// two normal pairs by Box-Muller with u = (x + 1/2) 2^-32.  Normals 2e and
// 2e + 1 weight element e = y N + x; normals 2 N^2 + 2s, + 1 weight
// subharmonic s = 8 (level - 1) + k, k over the 8 neighbours (iy, ix) of the
// origin in the order iy, ix = -1, 0, 1.
//
// One workgroup takes screen pairs j = blockIdx.x, + gridDim.x, ...; per
// pair the screens' transform is made once, and per screen: field = pupil
// exp(i phi) -> FFT -> |.|^2 (PSF) -> FFT (OTF) -> normalised by OTF(0),
// accumulated over the half plane of frequencies.  The second screen's
// phases over the pupil's bounding box wait in LDS while the first screen
// is used.
// The transforms leave their output in the storage order of fft2d_lds;
// element-wise steps work there, and each thread moves its pixels back to
// natural order through registers before the next transform.
#include "device_common.hpp"
#include "kernels.hpp"

#include <algorithm>

namespace nvsm {

namespace {

constexpr int ST = 512;

__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// The four normals of counter (j, w, m, 0).
__device__ __forceinline__ void normals4(uint32_t j, uint32_t w, uint32_t m, uint32_t k0, uint32_t k1,
                                         float (&g)[4]) {
    uint32_t c[4] = {j, w, m, 0u};
    philox4x32_10(c, k0, k1);
#pragma unroll
    for (int a = 0; a < 4; a += 2) {
        const float u1 = (float)(((double)c[a] + 0.5) * 0x1p-32);
        const float u2 = (float)(((double)c[a + 1] + 0.5) * 0x1p-32);
        const float r = sqrtf(-2.0f * logf(u1));
        float s, co;
        sincospif(2.0f * u2, &s, &co);
        g[a] = r * co;
        g[a + 1] = r * s;
    }
}

// Subharmonic s: level p = s / 8 + 1, neighbour k = s % 8 -> (iy, ix).
__device__ __forceinline__ void sub_offset(int k, int &iy, int &ix) {
    const int q = k < 4 ? k : k + 1;        // skip the centre of the 3 x 3 block
    iy = q / 3 - 1;
    ix = q % 3 - 1;
}

template <int N>
__global__ __launch_bounds__(ST) void k_stf(int pairs, float amp, const double *__restrict__ x_dev, uint32_t k0,
                                            uint32_t k1, uint32_t stream, const float2 *__restrict__ twiddle,
                                            float2 *__restrict__ part_a, float *__restrict__ part_s) {
    constexpr int P = LdsPitch<N>::v;
    constexpr int NP = (N / 2 + 1) * N;           // half plane: rows 0..N/2
    constexpr int PX = N * N / ST;                // pixels per thread
    constexpr int WD = N * N / 2 / ST;            // grid words per thread
    __shared__ float2 z[N * P];
    __shared__ float2 tw[N];
    __shared__ float2 sh[24];                     // subharmonic coefficients
    __shared__ float2 sct[3][N];                  // (cos, sin)(2 pi t / (N 3^p)), t = 0 .. N - 1
    constexpr int PB = N / 2, PB0 = N / 4;        // the pupil's bounding box: [PB0, PB0 + PB)^2
    __shared__ float side[PB * PB];               // the second screen's phases over that box
    const int tid = threadIdx.x;
    for (int i = tid; i < N; i += ST) tw[i] = twiddle[i];
    // the subharmonic phases depend on one coordinate and the level only:
    // formed once here (by the same calls the per-pixel form made)
    for (int i = tid; i < 3 * N; i += ST) {
        const int p = i / N + 1, t = i % N;
        const float inv = 1.0f / ((float)N * (p == 1 ? 3.f : p == 2 ? 9.f : 27.f));
        float sn, cs;
        sincospif(2.0f * (float)t * inv, &sn, &cs);
        sct[p - 1][t] = make_float2(cs, sn);
    }
    if (x_dev) {                                   // D/r0 from device memory: r0 = (N/2) / (D/r0) px
        const double r0 = (N / 2.0) / *x_dev;
        amp = (float)(0.15165750888103102 * pow(r0, -5.0 / 6.0) * pow((double)N, 5.0 / 6.0));   // sqrt(0.023)
    }

    // this workgroup's sums, kept in its own slice of the partials (each
    // thread always adds to the same entries, so no other thread touches them)
    float2 *pa = part_a + (size_t)blockIdx.x * NP;
    float *ps = part_s + (size_t)blockIdx.x * NP;
    for (int q = tid; q < NP; q += ST) {
        pa[q] = make_float2(0.f, 0.f);
        ps[q] = 0.f;
    }
    constexpr int PUPIL_R2 = (N / 2) * (N / 2);   // (2x - (N-1))^2 + (2y - (N-1))^2 <= (N/2)^2
    auto in_pupil = [](int y, int x) {
        const int dx = 2 * x - (N - 1), dy = 2 * y - (N - 1);
        return dx * dx + dy * dy <= PUPIL_R2;
    };

    // storage position -> natural index along one axis of the transform
    auto nat = [](int p) { return (p % FftGeom<N>::R1) * FftGeom<N>::R2 + p / FftGeom<N>::R1; };
    // A pair's screens are the real and imaginary parts of one transform:
    // the first screen's field goes to registers, the second screen's
    // phases inside the pupil to the side buffer, until its turn.
    for (int j = blockIdx.x; j < pairs; j += gridDim.x) {
        {
            __syncthreads();                       // previous use of z, sh and side done
            // spectrum of the screen pair, natural order
#pragma unroll 1
            for (int q = 0; q < WD; ++q) {
                const int w = q * ST + tid;        // elements 2w, 2w + 1 (same row)
                float g[4];
                normals4((uint32_t)j, (uint32_t)w, stream, k0, k1, g);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int e = 2 * w + h, y = e / N, x = e % N;
                    const int kx = x < N / 2 ? x : x - N, ky = y < N / 2 ? y : y - N;
                    const float f2 = (float)(kx * kx + ky * ky);
                    // sqrt(PSD(|k| / N)) / N = amp |k|^(-11/6), amp = sqrt(0.023) r0^(-5/6) N^(5/6)
                    const float sig = f2 > 0.f ? amp * exp2f((-11.0f / 12.0f) * log2f(f2)) : 0.f;
                    z[y * P + x] = make_float2(sig * g[2 * h], sig * g[2 * h + 1]);
                }
            }
            if (tid < 12) {
                float g[4];
                normals4((uint32_t)j, (uint32_t)(N * N / 2 + tid), stream, k0, k1, g);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int s = 2 * tid + h, p = s / 8 + 1;
                    const float t3 = p == 1 ? 3.f : p == 2 ? 9.f : 27.f;
                    int iy, ix;
                    sub_offset(s % 8, iy, ix);
                    // |f| = kk / N with kk = |(ix, iy)| / 3^p; sqrt(PSD) df / 3^p = amp kk^(-11/6) / 3^p
                    const float kk = sqrtf((float)(ix * ix + iy * iy)) / t3;
                    const float sig = amp * exp2f((-11.0f / 6.0f) * log2f(kk)) / t3;
                    sh[s] = make_float2(sig * g[2 * h], sig * g[2 * h + 1]);
                }
            }
            __syncthreads();
            fft2d_lds<N, ST>(z, tw);
            // subharmonics, in place at each stored position
#pragma unroll 1
            for (int i = tid; i < N * N; i += ST) {
                const int row = i / N, col = i % N;
                const int y = nat(row), x = nat(col);
                float2 v = z[row * P + col];
#pragma unroll
                for (int p = 1; p <= 3; ++p) {
                    // exp(2 pi i x / (N 3^p)) and the same for y
                    const float2 tx = sct[p - 1][x], ty = sct[p - 1][y];
                    const float cx = tx.x, sx = tx.y, cy = ty.x, sy = ty.y;
#pragma unroll
                    for (int kk = 0; kk < 8; ++kk) {
                        int iy, ix;
                        sub_offset(kk, iy, ix);
                        const float exr = ix ? cx : 1.f, exi = (float)ix * sx;     // exp(i ix a), ix in -1, 0, 1
                        const float eyr = iy ? cy : 1.f, eyi = (float)iy * sy;
                        const float er = exr * eyr - exi * eyi, ei = exr * eyi + exi * eyr;
                        const float2 c = sh[8 * (p - 1) + kk];
                        v.x += c.x * er - c.y * ei;
                        v.y += c.x * ei + c.y * er;
                    }
                }
                z[row * P + col] = v;
            }
            __syncthreads();
        }
        // field = pupil exp(i phi) of the first screen, to natural order; the
        // second screen's phases to the side buffer
        float2 t[PX];
#pragma unroll
        for (int k = 0; k < PX; ++k) {
            const int e = k * ST + tid, y = e / N, x = e % N;
            float s = 0.f, c = 0.f;
            if (in_pupil(y, x)) {
                const float2 v = z[fft_pos<N>(y) * P + fft_pos<N>(x)];
                sincosf(v.x, &s, &c);
                side[(y - PB0) * PB + (x - PB0)] = v.y;
            }
            t[k] = make_float2(c, s);
        }
        // (unrolled: the first screen's field is dead once in LDS, so it is
        // not held through the second screen's steps)
#pragma unroll
        for (int scr = 0; scr < 2; ++scr) {
            if (scr) {
#pragma unroll
                for (int k = 0; k < PX; ++k) {
                    const int e = k * ST + tid, y = e / N, x = e % N;
                    float s = 0.f, c = 0.f;
                    if (in_pupil(y, x)) sincosf(side[(y - PB0) * PB + (x - PB0)], &s, &c);
                    t[k] = make_float2(c, s);
                }
            }
            __syncthreads();                       // the transform (or the last OTF) was read
#pragma unroll
            for (int k = 0; k < PX; ++k) {
                const int e = k * ST + tid;
                z[(e / N) * P + e % N] = t[k];
            }
            __syncthreads();
            fft2d_lds<N, ST>(z, tw);
            // PSF = |.|^2, to natural order for the next transform
            float psf[PX];
#pragma unroll
            for (int k = 0; k < PX; ++k) {
                const int e = k * ST + tid, y = e / N, x = e % N;
                const float2 v = z[fft_pos<N>(y) * P + fft_pos<N>(x)];
                psf[k] = v.x * v.x + v.y * v.y;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < PX; ++k) {
                const int e = k * ST + tid;
                z[(e / N) * P + e % N] = make_float2(psf[k], 0.f);
            }
            __syncthreads();
            fft2d_lds<N, ST>(z, tw);
            const float o0 = z[0].x;               // OTF(0) = sum of the PSF
#pragma unroll 4
            for (int q = tid; q < NP; q += ST) {
                const int uy = q / N, ux = q % N;
                const float2 o = z[fft_pos<N>(uy) * P + fft_pos<N>(ux)];
                const float ox = o.x / o0, oy = o.y / o0;    // (a division: exactly 1 at u = 0)
                const float2 a = pa[q];
                pa[q] = make_float2(a.x + ox, a.y + oy);
                ps[q] += ox * ox + oy * oy;
            }
        }
    }
}

// Sums the workgroups' partials in FP64 and writes <|OTF|^2> (and <OTF>)
// over the full grid: the half plane directly, the other half from
// S(-u) = S(u) and <OTF>(-u) = conj <OTF>(u).
// Each workgroup takes 32 frequencies; 8 threads per frequency sum strided
// eighths of the workgroup partials, combined in a fixed order (so the sums
// are repeatable), which keeps 8 times as many loads in flight as one thread
// per frequency would.
constexpr int FIN_PARTS = 8, FIN_Q = 256 / FIN_PARTS;
template <int N>
__global__ __launch_bounds__(256) void k_stf_finalize(int nwg, double inv_screens, const float2 *__restrict__ part_a,
                                                      const float *__restrict__ part_s, double *__restrict__ stf,
                                                      double2 *__restrict__ mean_otf) {
    constexpr int NP = (N / 2 + 1) * N;
    __shared__ double red[3][FIN_PARTS][FIN_Q];
    const int lq = threadIdx.x % FIN_Q, part = threadIdx.x / FIN_Q;
    const int q = blockIdx.x * FIN_Q + lq;
    double ax = 0.0, ay = 0.0, s = 0.0;
    if (q < NP) {
        for (int b = part; b < nwg; b += FIN_PARTS) {
            const float2 a = part_a[(size_t)b * NP + q];
            ax += (double)a.x;
            ay += (double)a.y;
            s += (double)part_s[(size_t)b * NP + q];
        }
    }
    red[0][part][lq] = ax;
    red[1][part][lq] = ay;
    red[2][part][lq] = s;
    __syncthreads();
    if (part != 0 || q >= NP) return;
    ax = ay = s = 0.0;
#pragma unroll
    for (int k = 0; k < FIN_PARTS; ++k) {
        ax += red[0][k][lq];
        ay += red[1][k][lq];
        s += red[2][k][lq];
    }
    ax *= inv_screens;
    ay *= inv_screens;
    s *= inv_screens;
    const int uy = q / N, ux = q % N;
    stf[uy * N + ux] = s;
    if (mean_otf) mean_otf[uy * N + ux] = make_double2(ax, ay);
    if (uy >= 1 && uy < N / 2) {
        const int my = N - uy, mx = (N - ux) & (N - 1);
        stf[my * N + mx] = s;
        if (mean_otf) mean_otf[my * N + mx] = make_double2(ax, -ay);
    }
}

template <int N>
hipError_t launch_stf_t(const StfArgs &a, hipStream_t st) {
    hipLaunchKernelGGL((k_stf<N>), dim3(a.nwg), dim3(ST), 0, st, a.pairs, a.amp, a.x_dev, a.k0, a.k1, a.stream,
                       a.twiddle, a.part_a, a.part_s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    constexpr int NP = (N / 2 + 1) * N;
    hipLaunchKernelGGL((k_stf_finalize<N>), dim3((NP + FIN_Q - 1) / FIN_Q), dim3(256), 0, st, a.nwg, 1.0 / (2.0 * a.pairs),
                       a.part_a, a.part_s, a.stf, a.mean_otf);
    return hipGetLastError();
}

// Seeing fit of one cube per workgroup (FP64).  The frame-group sums of the
// box (see k_ratio) give m = <I> and P = <|I|^2>; the ratio
// eps = (|m|^2 - P/F) / (P (1 - 1/F)) is averaged over the annuli
// q - 1/2 <= |u| < q + 1/2 of the half plane (uy > 0, or uy = 0 < ux).  For
// each model point j the same annuli of
//   sum_k |w(k)|^2 P(u - k) rho_j(u - k) / sum_k |w(k)|^2 P(u - k),
// rho_j = |<OTF>|^2 / <|OTF|^2> (rho_j(0) left out; |w|^2 = 1/4, 1/16 per
// axis at offsets 0, +-1 with the taper, only k = 0 without) give the model
// curve; the cube's D/r0 minimises the squared distance (first minimum, then
// the vertex of the parabola through it and its neighbours, in grid index).
// Sums over annuli and candidates run in a fixed order.
template <int N>
__global__ __launch_bounds__(256) void k_seeing_fit(const SeeingFitArgs a) {
    constexpr int MAXE = (RATIO_MAX_BINS + 3) * (2 * RATIO_MAX_BINS + 5);
    __shared__ double mre[MAXE], mim[MAXE], pw[MAXE], val[MAXE];
    __shared__ double eq[RATIO_MAX_BINS], cq[RATIO_MAX_BINS];
    __shared__ double err[RATIO_MAX_POINTS];
    __shared__ int bin[MAXE];
    __shared__ int lst[MAXE];                 // the entries of each annulus, e ascending
    __shared__ int lo[RATIO_MAX_BINS + 1];    // annulus q: lst[lo[q - 1] .. lo[q])
    const int cube = blockIdx.x, tid = threadIdx.x;
    const int B = a.B, bw = 2 * B + 1, nbox = (B + 1) * bw, Q = a.Q, F = a.F;
    const double invF = 1.0 / F;
    for (int e = tid; e < nbox; e += 256) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int k = 0; k < a.nchunks; ++k) {
            const float *pp = a.part + ((size_t)(cube * a.nchunks + k) * nbox + e) * 3;
            s0 += (double)pp[0];
            s1 += (double)pp[1];
            s2 += (double)pp[2];
        }
        mre[e] = s0 * invF;
        mim[e] = s1 * invF;
        pw[e] = s2 * invF;
        // annulus of the entry (the half plane only), 0 if none; formed once
        // here, since the annulus means of every model point scan it
        const int uy = e / bw, ux = e % bw - B;
        int q = 0;
        if (!(uy == 0 && ux <= 0)) {
            q = (int)floor(sqrt((double)(uy * uy + ux * ux)) + 0.5);
            if (q > Q) q = 0;
        }
        bin[e] = q;
    }
    __syncthreads();
    // the annulus lists: counts, offsets, then each annulus's entries in
    // ascending order (so the annulus means add in the order of a plain scan)
    if (tid < Q) {
        int c = 0;
        for (int e = 0; e < nbox; ++e) c += bin[e] == tid + 1;
        lo[tid + 1] = c;
    }
    __syncthreads();
    if (tid == 0) {
        lo[0] = 0;
        for (int q = 1; q <= Q; ++q) lo[q] += lo[q - 1];
    }
    __syncthreads();
    if (tid < Q) {
        int k = lo[tid];
        for (int e = 0; e < nbox; ++e)
            if (bin[e] == tid + 1) lst[k++] = e;
    }
    __syncthreads();
    // mean of val over annulus tid + 1 (threads tid < Q)
    auto annulus_mean = [&]() {
        double sum = 0.0;
        for (int k = lo[tid]; k < lo[tid + 1]; ++k) sum += val[lst[k]];
        return sum / (lo[tid + 1] - lo[tid]);
    };
    // P at (vy, vx), |vx| <= B, -1 <= vy <= B (P(-v) = P(v))
    auto p_at = [&](int vy, int vx) {
        if (vy < 0) { vy = -vy; vx = -vx; }
        return pw[vy * bw + vx + B];
    };
    for (int e = tid; e < nbox; e += 256) {
        double v = 0.0;
        if (bin[e]) {
            const double m2 = mre[e] * mre[e] + mim[e] * mim[e], P = pw[e];
            v = P > 0.0 ? (m2 - P * invF) / (P * (1.0 - invF)) : 0.0;
        }
        val[e] = v;
    }
    __syncthreads();
    if (tid < Q) {
        eq[tid] = annulus_mean();
        if (a.curves) a.curves[(size_t)cube * Q + tid] = eq[tid];
    }
    __syncthreads();
    const int kr = a.window ? 1 : 0;
    for (int j = 0; j < a.J; ++j) {
        const double *S = a.tab_s + (size_t)j * N * N;
        const double2 *A = a.tab_a + (size_t)j * N * N;
        for (int e = tid; e < nbox; e += 256) {
            double v = 0.0;
            if (bin[e]) {
                const int uy = e / bw, ux = e % bw - B;
                double num = 0.0, den = 0.0;
                for (int ky = -kr; ky <= kr; ++ky)
                    for (int kx = -kr; kx <= kr; ++kx) {
                        const int vy = uy - ky, vx = ux - kx;
                        if (vy == 0 && vx == 0) continue;
                        const double wt = (kr ? (ky ? 0.0625 : 0.25) * (kx ? 0.0625 : 0.25) : 1.0) * p_at(vy, vx);
                        const int g = (vy & (N - 1)) * N + (vx & (N - 1));
                        const double sv = S[g];
                        const double2 av = A[g];
                        num += wt * (sv > 0.0 ? (av.x * av.x + av.y * av.y) / sv : 0.0);
                        den += wt;
                    }
                v = den > 0.0 ? num / den : 0.0;
            }
            val[e] = v;
        }
        __syncthreads();
        if (tid < Q) cq[tid] = annulus_mean();
        __syncthreads();
        if (tid == 0) {
            double e2 = 0.0;
            for (int q = 0; q < Q; ++q) e2 += (eq[q] - cq[q]) * (eq[q] - cq[q]);
            err[j] = e2;
        }
        __syncthreads();
    }
    if (tid == 0) {
        int jm = 0;
        for (int j = 1; j < a.J; ++j)
            if (err[j] < err[jm]) jm = j;
        double t = jm;
        if (jm > 0 && jm < a.J - 1) {
            const double den = err[jm - 1] - 2.0 * err[jm] + err[jm + 1];
            if (den > 0.0) t = jm + 0.5 * (err[jm - 1] - err[jm + 1]) / den;
        }
        a.x[1 + cube] = a.lo * pow(a.hi / a.lo, t / (a.J - 1.0));
    }
}

// D / <r0> = 1 / <1 / (D/r0)> over the cubes, into x[0].
__global__ void k_seeing_mean(int cubes, double *x) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int c = 0; c < cubes; ++c) s += 1.0 / x[1 + c];
        x[0] = cubes / s;
    }
}

}  // namespace

hipError_t launch_seeing_fit(const SeeingFitArgs &a, hipStream_t st) {
    if (a.cubes < 1 || a.Q < 2 || a.Q > RATIO_MAX_BINS || a.B != a.Q + 2 || a.J < 3 || a.J > RATIO_MAX_POINTS ||
        a.F < 2 || a.nchunks < 1)
        return hipErrorInvalidValue;
    if (a.N == 128)
        hipLaunchKernelGGL((k_seeing_fit<128>), dim3(a.cubes), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_seeing_fit<64>), dim3(a.cubes), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_seeing_mean, dim3(1), dim3(64), 0, st, a.cubes, a.x);
    return hipGetLastError();
}

hipError_t launch_stf(const StfArgs &a, hipStream_t st) {
    if (a.pairs < 1 || a.nwg < 1) return hipErrorInvalidValue;
    return a.N == 128 ? launch_stf_t<128>(a, st) : launch_stf_t<64>(a, st);
}

}  // namespace nvsm
