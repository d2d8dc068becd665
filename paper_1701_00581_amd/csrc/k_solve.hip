// Fourier modulus (Eq. 1) and phase (speckle-masking recursion), FP64.
//
// One workgroup per patch.  The phasors e(w) of the whole half disk live in
// LDS.  Frequencies are visited shell by shell (|w|^2 ascending); every w
// of a shell reads only strictly shorter frequencies, so a shell's w are
// independent: wave j takes the shell's w number j and j + 8, its lanes
// split that w's bispectrum samples, and a wave reduction gives
//   z(w) = sum_v e(w - v) e(v) conj B(w, v),  e(w) = z / |z|.
// The samples of the next shell are loaded into registers while the current
// shell is computed, so only LDS latency sits on the dependency chain.
#include "device_common.hpp"
#include "kernels.hpp"

namespace nvsm {

namespace {

constexpr int NT = 512;
constexpr int NWAVE = NT / 64;
constexpr int MAXW_PER_SHELL_WAVE = 2;   // up to 16 w per shell
constexpr int DEPTH = 4;                 // shells of samples in flight

template <int N> struct MaxW;
template <> struct MaxW<64> { static constexpr int v = 1504; };
template <> struct MaxW<128> { static constexpr int v = 6232; };

__device__ __forceinline__ double2 unit_or_one(double2 z) {
    const double m = sqrt(z.x * z.x + z.y * z.y);
    if (m == 0.0) return make_double2(1.0, 0.0);
    return make_double2(z.x / m, z.y / m);
}

template <int TPL>
struct ShellRegs {
    int w[MAXW_PER_SHELL_WAVE];
    int cnt[MAXW_PER_SHELL_WAVE];
    unsigned code[MAXW_PER_SHELL_WAVE][TPL];
    float2 b[MAXW_PER_SHELL_WAVE][TPL];
};

template <int N, int TPL>
__global__ __launch_bounds__(NT) void k_solve(int nW, int nshell, const int *__restrict__ shell_wb,
                                              const int *__restrict__ woff, const unsigned *__restrict__ code,
                                              const int *__restrict__ Wxy, const float *__restrict__ power,
                                              const float *__restrict__ mean_spec,
                                              const float2 *__restrict__ bispec, int64_t s_count,
                                              const double *__restrict__ stf, double floor_, int noise_bias,
                                              double *__restrict__ amp, double2 *__restrict__ phasor) {
    __shared__ double2 e[MaxW<N>::v];
    __shared__ double red[NWAVE];
    const int patch = blockIdx.x;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const float *P = power + (size_t)patch * N * N;

    // noise level: mean power where |u| > N/2 + 2 (signed u in [-N/2, N/2))
    double nb = 0.0;
    if (noise_bias) {
        double acc = 0.0;
        int cnt = 0;
        const double lim = (N / 2 + 2.0) * (N / 2 + 2.0);
        for (int j = tid; j < N * N; j += NT) {
            int ux = j % N, uy = j / N;
            ux = ux >= N / 2 ? ux - N : ux;
            uy = uy >= N / 2 ? uy - N : uy;
            if ((double)(ux * ux + uy * uy) > lim) { acc += (double)P[j]; ++cnt; }
        }
        acc = wave_sum_d(acc);
        double c = wave_sum_d((double)cnt);
        if (lane == 0) red[wave] = acc;
        __syncthreads();
        double tot = 0.0;
        for (int k = 0; k < NWAVE; ++k) tot += red[k];
        __syncthreads();
        if (lane == 0) red[wave] = c;
        __syncthreads();
        double ctot = 0.0;
        for (int k = 0; k < NWAVE; ++k) ctot += red[k];
        nb = tot / ctot;
    }
    // modulus, Eq. 1
    for (int i = tid; i < nW; i += NT) {
        const int wx = Wxy[2 * i], wy = Wxy[2 * i + 1];
        const int j = (wy & (N - 1)) * N + (wx & (N - 1));
        const double s = stf[j];
        double a = 0.0;
        if (s >= floor_) {
            const double num = (double)P[j] - nb;
            a = sqrt((num > 0.0 ? num : 0.0) / s);
        }
        amp[(size_t)patch * nW + i] = a;
    }
    // seeds (1,0) and (0,1) are W[0] and W[1]
    if (tid == 0) {
        const float *m = mean_spec + (size_t)patch * 4;
        e[0] = unit_or_one(make_double2((double)m[0], (double)m[1]));
        e[1] = unit_or_one(make_double2((double)m[2], (double)m[3]));
    }

    const float2 *B = bispec + (size_t)patch * s_count;
    // Loads are issued unconditionally (clamped to entry 0 where there is no
    // sample) so that every shell issues the same number of loads.
    auto load = [&](int s, ShellRegs<TPL> &r) __attribute__((always_inline)) {
        const int wb = shell_wb[s], nw = shell_wb[s + 1] - wb;
#pragma unroll
        for (int m = 0; m < MAXW_PER_SHELL_WAVE; ++m) {
            const int jj = wave + NWAVE * m;
            const bool has = jj < nw;
            const int w = has ? wb + jj : 0;
            const int o = woff[w], cnt = has ? woff[w + 1] - o : 0;
            r.w[m] = has ? w : -1;
            r.cnt[m] = cnt;
#pragma unroll
            for (int i = 0; i < TPL; ++i) {
                const int t = lane + 64 * i;
                const int idx = t < cnt ? o + t : 0;
                r.code[m][i] = code[idx];
                r.b[m][i] = B[idx];
            }
        }
    };
    auto solve = [&](const ShellRegs<TPL> &r) __attribute__((always_inline)) {
#pragma unroll
        for (int m = 0; m < MAXW_PER_SHELL_WAVE; ++m) {
            if (r.w[m] >= 0) {
                double zx = 0.0, zy = 0.0;
#pragma unroll
                for (int i = 0; i < TPL; ++i) {
                    const int t = lane + 64 * i;
                    if (t < r.cnt[m]) {
                        const unsigned cd = r.code[m][i];
                        const unsigned ia = cd >> 16, ib = cd & 0xffffu;
                        double2 ea = e[ia & 0x7fffu];
                        double2 eb = e[ib & 0x7fffu];
                        if (ia & 0x8000u) ea.y = -ea.y;
                        if (ib & 0x8000u) eb.y = -eb.y;
                        const double px = ea.x * eb.x - ea.y * eb.y;
                        const double py = ea.x * eb.y + ea.y * eb.x;
                        const double bx = (double)r.b[m][i].x, by = (double)r.b[m][i].y;
                        // (px + i py) * conj(bx + i by)
                        zx += px * bx + py * by;
                        zy += py * bx - px * by;
                    }
                }
                zx = wave_sum_d(zx);
                zy = wave_sum_d(zy);
                if (lane == 0) e[r.w[m]] = unit_or_one(make_double2(zx, zy));
            }
        }
    };

    __syncthreads();
    // shells 1.. in order; the samples of shell s + DEPTH - 1 are loaded
    // while shell s is solved (a ring of DEPTH register sets)
    ShellRegs<TPL> ring[DEPTH];
#pragma unroll
    for (int d = 0; d < DEPTH - 1; ++d)
        if (1 + d < nshell) load(1 + d, ring[d]);
    for (int s0 = 1; s0 < nshell; s0 += DEPTH) {
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) {
            const int s = s0 + d;
            if (s < nshell) {
                if (s + DEPTH - 1 < nshell) load(s + DEPTH - 1, ring[(d + DEPTH - 1) % DEPTH]);
                solve(ring[d]);
                __syncthreads();
            }
        }
    }
    for (int i = tid; i < nW; i += NT) phasor[(size_t)patch * nW + i] = e[i];
}

template <int N, int TPL>
hipError_t launch_solve_t(const SolveArgs &a, hipStream_t st) {
    hipLaunchKernelGGL((k_solve<N, TPL>), dim3(a.patches), dim3(NT), 0, st, a.nW, a.nshell, a.shell_wb,
                       a.woff, a.code, a.Wxy, a.power, a.mean_spec, a.bispec, a.s_count, a.stf, a.floor,
                       a.noise_bias, a.amp, a.phasor);
    return hipGetLastError();
}

template <int N>
hipError_t launch_solve_n(const SolveArgs &a, hipStream_t st) {
    if (a.max_sw <= 128) return launch_solve_t<N, 2>(a, st);
    if (a.max_sw <= 256) return launch_solve_t<N, 4>(a, st);
    return launch_solve_t<N, 8>(a, st);
}

}  // namespace

hipError_t launch_solve(const SolveArgs &a, hipStream_t st) {
    if (a.patches == 0) return hipSuccess;
    if (a.max_sw > 512 || a.nW > (a.N == 128 ? MaxW<128>::v : MaxW<64>::v)) return hipErrorInvalidValue;
    return a.N == 128 ? launch_solve_n<128>(a, st) : launch_solve_n<64>(a, st);
}

}  // namespace nvsm
