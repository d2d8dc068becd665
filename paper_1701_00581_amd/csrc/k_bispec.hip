// Bispectrum accumulation B(w, v) = <I(w - v) I(v) conj I(w)> over the
// frames of the burst (speckle masking; the hot loop of the path).
//
// Work decomposition (see plan.cpp): a workgroup owns one patch and one
// work item = an 8x8 block of w (one w per lane) times up to 4 x 32 values
// of v (one v per wave slot, the same for all 64 lanes).  Per frame:
//   * the region of I holding every w - v of the item, the slot values
//     I(v) and the block's I(w) are staged in LDS, GF frames at a time,
//     double buffered (the next group is fetched while this one is used);
//   * each slot costs one LDS gather, half a broadcast read and 8 FP32
//     FMA/MUL per lane.
// Accumulators stay in registers for the whole burst: a plain FP32 sum over
// KB frames, folded into a Kahan (sum, compensation) pair every KB frames.
#include "device_common.hpp"
#include "kernels.hpp"
#include "plan.hpp"

#include <cstdlib>

namespace nvsm {

namespace {

constexpr int NT = BS_WAVES * 64;
constexpr int KB = 20;                     // frames per compensated block

// LDS staging record of one frame: the item's region of I (w - v values),
// then the slot values I(v) of the 4 waves, then the 64 I(w) of the block.
template <int K> struct Stage {
    static constexpr int RMAX = bs_region_cap(K);               // padded region extent
    static constexpr int NV = BS_WAVES * K;
    static constexpr int SZ = RMAX + NV + 64 + 1;               // float2 per frame (+1 sink)
    static constexpr int PER = (RMAX + NV + 64 + NT - 1) / NT;  // loads per thread per frame
};

template <int N, int K, int GF>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(K <= 16 ? 3 : 2))) void k_bispec(
    const float2 *__restrict__ spec, int F, int n_items, int total, const int *__restrict__ items,
    const int *__restrict__ slot, const int *__restrict__ out_idx, float2 *__restrict__ bispec,
    int64_t s_count, float invF) {
    constexpr int HALF = N / 2;
    using St = Stage<K>;
    __shared__ float2 lds[2 * GF * St::SZ];

    const int L = xcd_remap(blockIdx.x, total);
    const int patch = L / n_items, g = L % n_items;
    const int *it = items + g * BS_ITEM_INTS;
    const int bx0 = it[0], by0 = it[1], rx0 = it[2], ry0 = it[3], rw = it[4], npts = it[6];
    const int pitch = it[7], rext = pitch * it[5];   // LDS row pitch and extent of the region
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int ns = it[8 + wave];                      // slots of this wave
    const int wx = bx0 + (lane & 7), wy = by0 + (lane >> 3);
    const int lane_base = (wy - ry0) * pitch + (wx - rx0);
    const int *sl = slot + (size_t)(g * BS_WAVES + wave) * K * 2;

    int addr[K];
#pragma unroll
    for (int k = 0; k < K; ++k) addr[k] = lane_base - sl[2 * k];

    // The values this thread stages every frame: offsets in the frame's
    // stored spectrum record (always inside it; region points beyond the
    // stored rows are never used by a sample and read a clamped row) and
    // byte offsets in the LDS record (the last slot of the record is a sink
    // for threads with nothing to stage).  32-bit byte offsets on a uniform
    // frame base let the loads use scalar-base addressing.
    constexpr int FS = SpecRows<N>::FS;
    const int nstage = npts + St::NV + 64;
    int src[St::PER], dst[St::PER];
#pragma unroll
    for (int j = 0; j < St::PER; ++j) {
        const int i = tid + NT * j;
        int so = 0, d = St::SZ - 1;
        if (i < npts) {
            const int ix = i % rw, iy = i / rw, x = rx0 + ix;
            const int y = min(ry0 + iy, HALF - 1);
            so = (y + SPEC_NEG_ROWS) * N + (x & (N - 1));
            d = iy * pitch + ix;
        } else if (i < npts + St::NV) {
            so = slot[((size_t)(g * BS_WAVES) * K + (i - npts)) * 2 + 1];
            d = rext + (i - npts);
        } else if (i < nstage) {
            const int l = i - npts - St::NV;
            so = (by0 + (l >> 3) + SPEC_NEG_ROWS) * N + ((bx0 + (l & 7)) & (N - 1));
            d = rext + St::NV + l;
        }
        src[j] = so * (int)sizeof(float2);
        dst[j] = d * (int)sizeof(float2);
    }

    const float2 *sp = spec + (size_t)patch * F * FS;
    auto fetch = [&](int f0, float2 (&v)[GF][St::PER]) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < GF; ++q) {
            const gptr_c sf = uniform_ptr(sp + (size_t)min(f0 + q, F - 1) * FS);
#pragma unroll
            for (int j = 0; j < St::PER; ++j) v[q][j] = load_global_f2(sf, (unsigned)src[j]);
        }
    };
    auto store = [&](int buf, const float2 (&v)[GF][St::PER]) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < GF; ++q)
#pragma unroll
            for (int j = 0; j < St::PER; ++j)
                *(float2 *)((char *)(lds + (buf * GF + q) * St::SZ) + dst[j]) = v[q][j];
    };

    float2 t[K], s[K], c[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        t[k] = make_float2(0.f, 0.f);
        s[k] = make_float2(0.f, 0.f);
        c[k] = make_float2(0.f, 0.f);
    }

    {
        float2 v[GF][St::PER];
        fetch(0, v);
        store(0, v);
    }
    __syncthreads();

    // Every slot is computed (slots past this wave's count hold a valid v
    // of the item and their results are dropped), so the frame is one
    // branch-free block and its LDS reads can be issued ahead.
    auto one_frame = [&](const float2 *rg, int f) __attribute__((always_inline)) {
        const float2 cw = rg[rext + St::NV + lane];
        const float2 *vrow = rg + rext + wave * K;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float2 bv = vrow[k];
            const float2 a = rg[addr[k]];
            // p = I(w - v) I(v);  t += p conj I(w), as one FMA chain
            const float pr = fmaf(a.x, bv.x, -(a.y * bv.y));
            const float pi = fmaf(a.x, bv.y, a.y * bv.x);
            t[k].x = fmaf(pr, cw.x, fmaf(pi, cw.y, t[k].x));
            t[k].y = fmaf(pi, cw.x, fmaf(-pr, cw.y, t[k].y));
        }
        if ((f + 1) % KB == 0 || f + 1 == F) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                kahan_add(s[k].x, c[k].x, t[k].x);
                kahan_add(s[k].y, c[k].y, t[k].y);
                t[k] = make_float2(0.f, 0.f);
            }
        }
    };
    auto group = [&](int f0, auto bufc) __attribute__((always_inline)) {
        constexpr int BUF = decltype(bufc)::value;
        float2 nxt[GF][St::PER];
        const bool more = f0 + GF < F;
        if (more) fetch(f0 + GF, nxt);
#pragma unroll
        for (int q = 0; q < GF; ++q)
            if (f0 + q < F) one_frame(lds + (BUF * GF + q) * St::SZ, f0 + q);
        if (more) store(1 - BUF, nxt);
        __syncthreads();
    };

    for (int f = 0; f < F; f += 2 * GF) {
        group(f, std::integral_constant<int, 0>{});
        if (f + GF < F) group(f + GF, std::integral_constant<int, 1>{});
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
    static const int gf = [] {
        const char *e = getenv("NVSM_BISPEC_GF");
        int v = e ? atoi(e) : 1;
        return (v == 1 || v == 2 || v == 4) ? v : 1;
    }();
#define NVSM_LAUNCH_BS(NN, KK, GG)                                                                          \
    hipLaunchKernelGGL((k_bispec<NN, KK, GG>), dim3(total), dim3(NT), 0, st, a.spectra, a.F, a.n_items, total, \
                       a.items, a.slot_v, a.out_idx, a.bispec, a.s_count, 1.0f / a.F)
#define NVSM_LAUNCH_G(NN, KK)                                                                   \
    if (gf == 1) NVSM_LAUNCH_BS(NN, KK, 1); else if (gf == 2) NVSM_LAUNCH_BS(NN, KK, 2); else NVSM_LAUNCH_BS(NN, KK, 4);
    if (a.slots == 16) {
        if (a.N == 128) { NVSM_LAUNCH_G(128, 16) } else { NVSM_LAUNCH_G(64, 16) }
    } else if (a.slots == 24) {
        if (a.N == 128) { NVSM_LAUNCH_G(128, 24) } else { NVSM_LAUNCH_G(64, 24) }
    } else {
        return hipErrorInvalidValue;
    }
#undef NVSM_LAUNCH_G
#undef NVSM_LAUNCH_BS
    return hipGetLastError();
}

}  // namespace nvsm
