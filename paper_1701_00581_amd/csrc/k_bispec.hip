// Bispectrum accumulation B(w, v) = <I(w - v) I(v) conj I(w)> over the
// frames of the burst (speckle masking; the hot loop of the path).
//
// Work decomposition (see plan.cpp): a workgroup owns one patch and one
// work item = an 8x8 block of w (one w per lane) times up to 4 x 32 values
// of v (one v per wave slot, the same for all 64 lanes).  Per frame:
//   * the region of I holding every w - v of the item is staged in LDS
//     (double buffered; frame f+1 is fetched while frame f is computed);
//   * I(w) comes from the stored spectrum (one value per lane);
//   * I(v) is wave-uniform and comes through the scalar cache;
//   * each slot costs one LDS read and 8 FP32 FMA/MUL per lane.
// Accumulators stay in registers for the whole burst: a plain FP32 sum over
// KB frames, folded into a Kahan (sum, compensation) pair every KB frames.
#include "device_common.hpp"
#include "kernels.hpp"
#include "plan.hpp"

namespace nvsm {

namespace {

constexpr int NT = BS_WAVES * 64;
constexpr int MAXP = BS_MAX_REGION / NT;   // staged points per thread
constexpr int KB = 8;                      // frames per compensated block

template <int N>
__global__ __launch_bounds__(NT) void k_bispec(const float2 *__restrict__ spec, int F, int n_items,
                                               int total, const int *__restrict__ items,
                                               const int *__restrict__ slot, const int *__restrict__ out_idx,
                                               float2 *__restrict__ bispec, int64_t s_count, float invF) {
    constexpr int HALF = N / 2;
    constexpr int FS = HALF * N;               // float2 per stored frame spectrum
    constexpr int K = BS_SLOTS;
    __shared__ float2 reg[2 * BS_MAX_REGION];

    const int L = xcd_remap(blockIdx.x, total);
    const int patch = L / n_items, g = L % n_items;
    const int *it = items + g * BS_ITEM_INTS;
    const int bx0 = it[0], by0 = it[1], rx0 = it[2], ry0 = it[3], rw = it[4], npts = it[6];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int ns = it[8 + wave];
    const int wx = bx0 + (lane & 7), wy = by0 + (lane >> 3);
    const int lane_base = (wy - ry0) * rw + (wx - rx0);
    const int *sl = slot + (size_t)(g * BS_WAVES + wave) * K * 2;

    int addr[K];
#pragma unroll
    for (int k = 0; k < K; ++k) addr[k] = lane_base - sl[2 * k];

    // where each staged point comes from (bit 31: conjugate; -1: outside
    // the stored rows, staged as 0 and never used by a valid sample)
    int src[MAXP];
#pragma unroll
    for (int j = 0; j < MAXP; ++j) {
        const int i = tid + NT * j;
        int s = -1;
        if (i < npts) {
            const int x = rx0 + i % rw, y = ry0 + i / rw;
            if (y >= 0 && y < HALF) s = y * N + (x & (N - 1));
            else if (y < 0 && -y < HALF) s = (int)((unsigned)((-y) * N + ((-x) & (N - 1))) | 0x80000000u);
        }
        src[j] = s;
    }

    const float2 *sp = spec + (size_t)patch * F * FS;
    auto fetch = [&](int f, float2 *dst) {
        const float2 *sf = sp + (size_t)f * FS;
#pragma unroll
        for (int j = 0; j < MAXP; ++j) {
            float2 v = make_float2(0.f, 0.f);
            const int s = src[j];
            if (s != -1) {
                v = sf[s & 0x7fffffff];
                if (s < 0) v.y = -v.y;
            }
            dst[j] = v;
        }
    };
    auto store = [&](int buf, const float2 *v) {
#pragma unroll
        for (int j = 0; j < MAXP; ++j) {
            const int i = tid + NT * j;
            if (i < npts) reg[buf * BS_MAX_REGION + i] = v[j];
        }
    };

    float2 t[K], s[K], c[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        t[k] = make_float2(0.f, 0.f);
        s[k] = make_float2(0.f, 0.f);
        c[k] = make_float2(0.f, 0.f);
    }

    {
        float2 v[MAXP];
        fetch(0, v);
        store(0, v);
    }
    __syncthreads();

    auto frame = [&](int f, auto bufc) {
        constexpr int BUF = decltype(bufc)::value;
        const float2 *sf = sp + (size_t)f * FS;
        float2 nxt[MAXP];
        const bool more = f + 1 < F;
        if (more) fetch(f + 1, nxt);
        const float2 cw = sf[wy * N + (wx & (N - 1))];
        const float2 *rg = reg + BUF * BS_MAX_REGION;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (k < ns) {
                const unsigned so = (unsigned)sl[2 * k + 1];
                float2 bv = sf[so & 0x7fffffffu];
                bv.y = __uint_as_float(__float_as_uint(bv.y) ^ (so & 0x80000000u));
                const float2 a = rg[addr[k]];
                const float tr = a.x * bv.x - a.y * bv.y;
                const float ti = a.x * bv.y + a.y * bv.x;
                t[k].x += tr * cw.x + ti * cw.y;
                t[k].y += ti * cw.x - tr * cw.y;
            }
        }
        if ((f + 1) % KB == 0 || f + 1 == F) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                kahan_add(s[k].x, c[k].x, t[k].x);
                kahan_add(s[k].y, c[k].y, t[k].y);
                t[k] = make_float2(0.f, 0.f);
            }
        }
        if (more) store(1 - BUF, nxt);
        __syncthreads();
    };

    for (int f = 0; f < F; f += 2) {
        frame(f, std::integral_constant<int, 0>{});
        if (f + 1 < F) frame(f + 1, std::integral_constant<int, 1>{});
    }

    const int *oi = out_idx + (size_t)(g * BS_WAVES + wave) * K * 64 + lane;
    float2 *bo = bispec + (size_t)patch * s_count;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (k < ns) {
            const int o = oi[k * 64];
            if (o >= 0) bo[o] = make_float2((s[k].x - c[k].x) * invF, (s[k].y - c[k].y) * invF);
        }
    }
}

}  // namespace

hipError_t launch_bispec(const BispecArgs &a, hipStream_t st) {
    const int total = a.patches * a.n_items;
    if (total == 0) return hipSuccess;
    if (a.N == 128)
        hipLaunchKernelGGL(k_bispec<128>, dim3(total), dim3(NT), 0, st, a.spectra, a.F, a.n_items, total,
                           a.items, a.slot_v, a.out_idx, a.bispec, a.s_count, 1.0f / a.F);
    else
        hipLaunchKernelGGL(k_bispec<64>, dim3(total), dim3(NT), 0, st, a.spectra, a.F, a.n_items, total,
                           a.items, a.slot_v, a.out_idx, a.bispec, a.s_count, 1.0f / a.F);
    return hipGetLastError();
}

}  // namespace nvsm
