// Bispectrum accumulation B(w, v) = <I(w - v) I(v) conj I(w)> over the
// frames of the burst (speckle masking; the hot loop of the path).
//
// Work decomposition (see plan.cpp): a workgroup owns one patch and one
// work item = a group of up to 64 w close in angle and radius (one w per
// lane) times 4 x NS values of v (one v per wave slot, the same for all 64
// lanes).  Per frame, and for the next frame while this one is computed:
//   * the region of I holding every w - v of the item goes to LDS by direct
//     16-byte global-to-LDS loads (no registers involved), double buffered;
//   * each lane loads its own I(w), and lane l the slot value I(v) of slot
//     l mod 16, into registers; a slot's value reaches every lane through a
//     DPP row broadcast folded into the multiplies that use it.
// Each slot then costs one 64-bit LDS gather and 8 FP32 FMA/MUL per lane.
// LDS bandwidth is the other limit of this loop (a 64-bit read returns 16
// lanes per clock), so I(v) and I(w) stay out of LDS and the lanes of a
// group are laid out for conflict-free gathers (see plan.cpp).
// Accumulators stay in registers for the whole burst: a plain FP32 sum over
// KB frames, folded into a compensated sum every KB frames (fold_carry).
#include "device_common.hpp"
#include "kernels.hpp"
#include "plan.hpp"

#include <algorithm>

namespace nvsm {

namespace {

constexpr int NT = BS_WAVES * 64;
constexpr int KB = 50;                     // frames per compensated block

// LDS record of one frame: the item's region of I (w - v values, row pitch =
// region width), moved in chunks of 128 complex values (one wave-wide
// 16-byte load each).
template <int K> struct Region {
    static constexpr int SZ = bs_max_region(K);                // float2 per frame
    static constexpr int CH = SZ / 128;                        // chunks per frame
    static constexpr int PERW = (CH + BS_WAVES - 1) / BS_WAVES;    // chunks per wave
    static_assert(SZ % 128 == 0, "region capacity must be whole chunks");
};

typedef __attribute__((address_space(3))) void *lds_ptr;
typedef unsigned u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned))));

__device__ __forceinline__ float2 as_f2(u32x2 v) { return make_float2(__uint_as_float(v[0]), __uint_as_float(v[1])); }

// b taken from lane K of this lane's row of 16 (DPP row_newbcast), times a
// (negated, for mul_bc_neg); and acc + that product.  Arithmetic only; EXEC
// must be full.
template <int K>
__device__ __forceinline__ float mul_bc(float b, float a) {
    float r;
    asm("v_mul_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "=v"(r) : "v"(b), "v"(a), "i"(K));
    return r;
}
template <int K>
__device__ __forceinline__ float mul_bc_neg(float b, float a) {
    float r;
    asm("v_mul_f32_dpp %0, -%1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "=v"(r) : "v"(b), "v"(a), "i"(K));
    return r;
}
template <int K>
__device__ __forceinline__ float fmac_bc(float acc, float b, float a) {
    asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "+v"(acc) : "v"(b), "v"(a), "i"(K));
    return acc;
}

// Compensated (Kahan) fold of the block sum t into s.  The rounding error
// of s + t, negated, is where the next block's sum starts: Kahan's
// correction travels in the next addend instead of a register of its own,
// so a slot holds two accumulators (s, t) rather than three.  The
// compensated total at any fold is s + t.
__device__ __forceinline__ void fold_carry(float &s, float &t) {
    const float u = s + t;
    t = t - (u - s);
    s = u;
}

// This lane's index in the wave.
__device__ __forceinline__ int lane_id() { return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// Waits until at most n vector-memory loads of this wave are in flight
// (they complete in order).
template <int n>
__device__ __forceinline__ void wait_vm() {
    static_assert(n >= 0 && n < 64, "vmcnt range");
    // s_waitcnt: vmcnt[3:0] | expcnt[6:4] = 7 | lgkmcnt[11:8] = 15 | vmcnt[5:4] at [15:14]
    __builtin_amdgcn_s_waitcnt((n & 15) | (7 << 4) | (15 << 8) | ((n >> 4) << 14));
}
// fn(integral_constant<k>) for k = 0 .. n - 1, unrolled at compile time.
template <int n, int k = 0, typename Fn>
__device__ __forceinline__ void static_for(Fn &&fn) {
    if constexpr (k < n) {
        fn(std::integral_constant<int, k>{});
        static_for<n, k + 1>(fn);
    }
}

// Waits until this wave's LDS reads are done: lgkmcnt(0), other counters free.
__device__ __forceinline__ void wait_lds() { __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (3 << 14)); }

// One work item with NS slots per wave (NS a multiple of 4, <= K).  Slots
// past a chunk's real v hold a valid v of the item; their results are
// dropped.  The frame's slot loop is one branch-free block, so its LDS reads
// can be issued ahead.
template <int N, int K, int NS, int MODE, int PERW>
__device__ __forceinline__ void bispec_item(float2 *lds0, float2 *lds1, const float2 *__restrict__ spec,
                                            int64_t rec0, int F, int patch, int g, const int *__restrict__ it,
                                            const int *__restrict__ group_xy, const int *__restrict__ slot,
                                            const int *__restrict__ out_idx, float2 *__restrict__ bispec,
                                            int64_t s_count, const AccState acc) {
    constexpr int HALF = N / 2;
    constexpr int FS = SpecRows<N>::FS;
    constexpr int FB = FS * (int)sizeof(float2);               // bytes per stored frame
    const int *gxy = group_xy + it[0] * (2 * BS_LANES);
    const int rx0 = it[1], ry0 = it[2], npts = it[5], pitch = it[6];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int wx = gxy[2 * lane], wy = gxy[2 * lane + 1];
    const int lane_base = (wy - ry0) * pitch + (wx - rx0);
    const int *sl = slot + (size_t)(g * BS_WAVES + wave) * K * 2;

    constexpr int NQ = (NS + 15) / 16;           // rows of 16 slot values
    int addr[NS];     // LDS byte offset of I(w - v) in the region, per slot
#pragma unroll
    for (int k = 0; k < NS; ++k) addr[k] = (lane_base - sl[2 * k]) * (int)sizeof(float2);
    int sol[NQ];      // byte offset of I(v) of slot 16 q + lane mod 16 in a frame's record
#pragma unroll
    for (int q = 0; q < NQ; ++q) sol[q] = sl[2 * min(16 * q + (lane & 15), K - 1) + 1] * (int)sizeof(float2);
    const int wo = ((wy + SPEC_NEG_ROWS) * N + (wx & (N - 1))) * (int)sizeof(float2);   // I(w)

    // Region staging: wave j moves chunks j, j + 4, ... of the region; lane
    // l of chunk c moves the complex values 128 c + 2 l and + 1.  The pitch
    // and the region's x0 are even (see plan.cpp), so each pair is one row,
    // two adjacent stored columns, 16-byte aligned.  src[] holds each lane's
    // byte offset in the frame's record: region points beyond the stored
    // rows are never used by a sample and read a clamped row; pairs past
    // the region read offset 0 into the unused tail of the LDS record.
    // PERW is the fewest chunks per wave that hold the item's region.
    // Every wave issues all PERW loads, so that their number is known when
    // the compiler places the waits for the loads issued before them.
    unsigned src[PERW];
#pragma unroll
    for (int j = 0; j < PERW; ++j) {
        const int e = 128 * (wave + BS_WAVES * j) + 2 * lane;
        int o = 0;
        if (e < npts) {
            const int ix = e % pitch, iy = e / pitch, x = rx0 + ix;
            const int y = min(ry0 + iy, HALF - 1);
            o = (y + SPEC_NEG_ROWS) * N + (x & (N - 1));
        }
        src[j] = (unsigned)(o * (int)sizeof(float2));
    }

    // the patch's spectra as one buffer resource; frame f at byte f * FB
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void *)(spec + (size_t)rec0 * FS), (short)0, F * FB, 0x00020000);
    // With the photon-noise terms, the last frame stages the same region of
    // the patch's C table (record layout) instead of a spare copy of itself,
    // so that the correction reads C(w - v) from LDS at the slots' offsets.
    const bool photon = MODE == 2 || (MODE == 1 && acc.noise_c != nullptr);
    const __amdgpu_buffer_rsrc_t rsrc_c = __builtin_amdgcn_make_buffer_rsrc(
        photon ? (void *)(acc.noise_c + (size_t)patch * FS) : (void *)spec, (short)0, photon ? FB : 0, 0x00020000);
    // the region loads of frame f into buf (f = F: the C table's region)
    auto fetch = [&](int f, float2 *buf) __attribute__((always_inline)) {
        const bool c = photon && f == F;
#pragma unroll
        for (int j = 0; j < PERW; ++j)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(c ? rsrc_c : rsrc, (lds_ptr)(buf + 128 * (wave + BS_WAVES * j)), 16,
                                                     (int)src[j], c ? 0 : f * FB, 0, 0);
    };
    auto load_vals = [&](int f, float2 &cw, float2 (&bv)[NQ]) __attribute__((always_inline)) {
        cw = as_f2(__builtin_amdgcn_raw_buffer_load_b64(rsrc, wo, f * FB, 0));
#pragma unroll
        for (int q = 0; q < NQ; ++q) bv[q] = as_f2(__builtin_amdgcn_raw_buffer_load_b64(rsrc, sol[q], f * FB, 0));
    };

    // running sums of earlier frame groups, in this launch's lane order:
    // slot k of lane l of wave j of item (patch, g) at
    // (((patch * n_items + g) * 4 + j) * K + k) * 64 + l
    // (wave-uniform base, so that only the lane offset needs a vector register)
    const size_t ls0 = (((size_t)patch * acc.n_items + g) * BS_WAVES + wave) * K * 64;
    // t: this block's sum (starting from the carried correction); s: the folded sum
    float2 t[NS], s[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        t[k] = make_float2(0.f, 0.f);
        s[k] = make_float2(0.f, 0.f);
    }
    if (MODE == 1 && !acc.first) {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            s[k] = acc.sum[ls0 + k * 64 + lane];
            const float2 c = acc.comp[ls0 + k * 64 + lane];
            t[k] = make_float2(-c.x, -c.y);
        }
    }

    float2 cw, bv[NQ];
    fetch(0, lds0);
    load_vals(0, cw, bv);
    wait_vm<0>();
    __builtin_amdgcn_s_barrier();

    // Frame f from LDS buffer rg with its values in cw, bv.  The next
    // frame's region goes to the other buffer meanwhile; its values replace
    // cw and bv once this frame's slot loop has used them.  Before the
    // barrier only the region loads are awaited (loads complete in order,
    // the 1 + NQ value loads were issued last).  Loads are issued without
    // branches, so the compiler knows how many are in flight at each use.
    auto frame = [&](int f, const float2 *rg, float2 *nxt) __attribute__((always_inline)) {
        // the last frame fetches itself again (unused) rather than branch, or
        // with the photon-noise terms the C region
        const int fn = min(f + 1, F - 1);
        fetch(photon ? f + 1 : fn, nxt);
        const char *rb = (const char *)rg;
        // p = I(w - v) I(v);  t += p conj I(w).  The gather of slot k + 1 is
        // requested before slot k is computed, so that its LDS latency runs
        // under slot k's arithmetic.
        float2 an = *(const float2 *)(rb + addr[0]);
        auto slot_k = [&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value, q = k / 16, r = k % 16;
            const float2 a = an;
            if constexpr (k + 1 < NS) an = *(const float2 *)(rb + addr[k + 1]);
            const float pr = fmac_bc<r>(mul_bc_neg<r>(bv[q].y, a.y), bv[q].x, a.x);
            const float pi = fmac_bc<r>(mul_bc<r>(bv[q].x, a.y), bv[q].y, a.x);
            t[k].x = fmaf(pr, cw.x, fmaf(pi, cw.y, t[k].x));
            t[k].y = fmaf(pi, cw.x, fmaf(pr, -cw.y, t[k].y));
        };
        static_for<NS>(slot_k);
        if ((f + 1) % KB == 0 || f + 1 == F) {
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                fold_carry(s[k].x, t[k].x);
                fold_carry(s[k].y, t[k].y);
            }
        }
        load_vals(fn, cw, bv);
        wait_vm<1 + NQ>();
        wait_lds();
        __builtin_amdgcn_s_barrier();
    };

    for (int f = 0; f < F; f += 2) {
        frame(f, lds0, lds1);
        if (f + 1 < F) frame(f + 1, lds1, lds0);
    }
    wait_vm<0>();

    if (MODE == 1 && acc.mode == 1) {
        // keep the running (sum, compensation) for the next frame group
        const int lane_e = lane_id();
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            acc.sum[ls0 + k * 64 + lane_e] = s[k];
            acc.comp[ls0 + k * 64 + lane_e] = make_float2(-t[k].x, -t[k].y);
        }
        return;
    }
    // (the lane index and 1/F are formed again here, so that neither keeps
    // a register through the frame loop)
    const int lane_e = lane_id();
    const int *oi = out_idx + (size_t)(g * BS_WAVES + wave) * K * 64 + lane_e;
    float2 *bo = bispec + (size_t)patch * s_count;
    const float inv = MODE == 1 ? acc.inv_total : 1.0f / (float)F;
    // (the streaming form's last group carries the photon-noise terms too)
    if (MODE == 2 || (MODE == 1 && acc.noise_c != nullptr)) {
        // (no fused multiply-adds here: both forms round these steps alike)
#pragma clang fp contract(off)
        // photon-noise terms: B -= C(w) + conj C(v) + conj C(w - v) - 2T,
        // C of the patch in the record layout of the spectra (the slot
        // table gives v's record index; w - v lies within the record's rows)
        // (w's row and column come from its record index, which stays live)
        const float2 *Cp = acc.noise_c + (size_t)patch * FS;
        const float t2 = 2.0f * acc.noise_t[(size_t)patch * 2 + 1];
        const int wi = wo / (int)sizeof(float2);
        // C(w - v) from the C region the last frame staged (in the buffer
        // after the last frame's)
        const char *cr = (const char *)((F & 1) ? lds1 : lds0);
        // the means first, so the block-sum registers are free for the loads
#pragma unroll
        for (int k = 0; k < NS; ++k) s[k] = make_float2((s[k].x + t[k].x) * inv, (s[k].y + t[k].y) * inv);
        const float2 c_w = Cp[wi];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const int vo = sl[2 * k + 1];
            const float2 c_v = Cp[vo];
            const float2 c_d = *(const float2 *)(cr + addr[k]);
            const int o = oi[k * 64];
            if (o >= 0)
                bo[o] = make_float2(s[k].x - (c_w.x + c_v.x + c_d.x - t2), s[k].y - (c_w.y - c_v.y - c_d.y));
        }
    } else {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const int o = oi[k * 64];
            if (o >= 0) bo[o] = make_float2((s[k].x + t[k].x) * inv, (s[k].y + t[k].y) * inv);
        }
    }
}

// Runs the item with its slot count (one of 4, 8, ..., Q * 4).
template <int N, int K, int Q, int MODE>
__device__ __forceinline__ void bispec_dispatch(int nq, float2 *lds0, float2 *lds1, const float2 *spec,
                                                int64_t rec0, int F, int patch, int g, const int *it, const int *group_xy,
                                                const int *slot, const int *out_idx, float2 *bispec,
                                                int64_t s_count, const AccState &acc) {
    if constexpr (Q > 0) {
        if (nq == Q) {
            // regions of up to half the capacity (most items) move half the chunks
            constexpr int PW = Region<K>::PERW, PH = PW > 1 ? PW / 2 : 1;
            if (it[5] <= 128 * BS_WAVES * PH)
                bispec_item<N, K, 4 * Q, MODE, PH>(lds0, lds1, spec, rec0, F, patch, g, it, group_xy, slot, out_idx,
                                                 bispec, s_count, acc);
            else
                bispec_item<N, K, 4 * Q, MODE, PW>(lds0, lds1, spec, rec0, F, patch, g, it, group_xy, slot, out_idx,
                                                 bispec, s_count, acc);
        } else
            bispec_dispatch<N, K, Q - 1, MODE>(nq, lds0, lds1, spec, rec0, F, patch, g, it, group_xy, slot, out_idx, bispec,
                                         s_count, acc);
    }
}

// Item L of the launch: (patch, work item) = (L / n_items, L % n_items).
template <int N, int K, int MODE>
__device__ __forceinline__ void bispec_one(int L, float2 *lds0, float2 *lds1, const BurstTable &bt,
                                           const float2 *spec, int n_items, const int *items, const int *group_xy,
                                           const int *slot, const int *out_idx, float2 *bispec, int64_t s_count,
                                           const AccState &acc) {
    const int patch = L / n_items, g = L % n_items;
    const int b = burst_of(bt, patch, [](const BurstDesc &d) { return (int64_t)d.patch0; });
    const int F = bt.b[b].F;
    const int64_t rec0 = bt.b[b].spec0 + (int64_t)(patch - bt.b[b].patch0) * F;
    const int *it = items + g * BS_ITEM_INTS;
    // this wave's slots / 4 (the waves of an item may differ; each runs the
    // same frame loop, so their barriers match)
    const int nq = __builtin_amdgcn_readfirstlane(it[8 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)]) >> 2;
    bispec_dispatch<N, K, K / 4, MODE>(nq, lds0, lds1, spec, rec0, F, patch, g, it, group_xy, slot, out_idx, bispec,
                                 s_count, acc);
}

// Item of position o in the launch order.  The order takes, for each XCD
// slot x = 0..7 in turn, slice x (an eighth of the patches) of every burst,
// so that the 8 contiguous ranges the XCDs work on (see xcd_remap) hold the
// same share of every burst even when the bursts' frame counts differ.
// With one burst it is the plain patch-major order.
__device__ __forceinline__ int item_at(const BurstTable &bt, int o, int n_items) {
    if (bt.nb == 1) return o;
    int ps = o / n_items;                      // patch position in the order
    const int g = o % n_items;
    for (int x = 0; x < 8; ++x)
        for (int b = 0; b < bt.nb; ++b) {
            const int P = (b + 1 < bt.nb ? bt.b[b + 1].patch0 : bt.patches) - bt.b[b].patch0;
            const int lo = P * x / 8, cnt = P * (x + 1) / 8 - lo;
            if (ps < cnt) return (bt.b[b].patch0 + lo + ps) * n_items + g;
            ps -= cnt;
        }
    return o;                                  // not reached: o < patches * n_items
}

// Waves per SIMD the kernel is built for.  With 16 slots it fits 96 VGPRs
// (two accumulators per slot value, 16 LDS offsets), i.e. 5 waves per
// SIMD; more waves hide more of the latency of the one LDS gather each slot
// waits for (measured: 51.7 ms at 5 waves against 53.6 ms at 4 with 97
// VGPRs, and 52.5 ms at 4 with all 16 gathers of a frame issued ahead; at 5
// waves a second gather in flight gains nothing).
// The photon form then keeps one 8-byte value in scratch across the frame
// loop (stored before it, reloaded after).  The persistent form
// (k_bispec_queue) needs about 100 VGPRs and runs at 4.
constexpr int bs_waves_per_eu(int K) { return K <= 16 ? 5 : 2; }

// One workgroup per item.  MODE 0 writes the mean of all frames; MODE 1
// adds a frame group to the running sums of acc (acc.mode 1 and 2); MODE 2
// writes the mean less the photon-noise terms of acc.noise_c/noise_t.  Each
// is a separate instantiation, so that the plain form carries none of the
// others' registers.
template <int N, int K, int MODE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(bs_waves_per_eu(K)))) void k_bispec(
    const BurstTable bt, const float2 *__restrict__ spec, int n_items, int total, const int *__restrict__ items,
    const int *__restrict__ group_xy, const int *__restrict__ slot, const int *__restrict__ out_idx,
    float2 *__restrict__ bispec, int64_t s_count, const AccState acc) {
    // two separate arrays, so that loads into one are known not to touch
    // the other
    __shared__ float2 lds0[Region<K>::SZ];
    __shared__ float2 lds1[Region<K>::SZ];
    bispec_one<N, K, MODE>(item_at(bt, xcd_remap(blockIdx.x, total), n_items), lds0, lds1, bt, spec, n_items, items,
                     group_xy, slot, out_idx, bispec, s_count, acc);
}

// Persistent form: as many workgroups as fit on the GPU at once, each
// taking items from a work queue until none is left.  The items are split
// into 8 contiguous ranges, one per XCD (workgroups are dispatched to the
// XCDs in turn, blockIdx mod 8), so that each XCD works on its own patches
// and keeps their spectra in its L2; a workgroup drains its own XCD's range
// first, then helps the others.  queue[8] counts the items taken from each
// range and must be zero at launch.  Every workgroup ends after finding all
// 8 ranges exhausted.
template <int N, int K, int MODE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(K <= 16 ? 4 : 2))) void k_bispec_queue(
    const BurstTable bt, const float2 *__restrict__ spec, int n_items, int total, const int *__restrict__ items,
    const int *__restrict__ group_xy, const int *__restrict__ slot, const int *__restrict__ out_idx,
    float2 *__restrict__ bispec, int64_t s_count, const AccState acc, int *__restrict__ queue) {
    __shared__ float2 lds0[Region<K>::SZ];
    __shared__ float2 lds1[Region<K>::SZ];
    __shared__ int next;
    const int x = blockIdx.x & 7;
    for (int k = 0; k < 8; ++k) {
        const int q = (x + k) & 7;
        const int beg = (int)((int64_t)total * q / 8);
        const int cnt = (int)((int64_t)total * (q + 1) / 8) - beg;
        for (;;) {
            __syncthreads();                     // the last item is done with LDS and `next`
            if (threadIdx.x == 0) next = atomicAdd(&queue[q], 1);
            __syncthreads();
            const int i = __builtin_amdgcn_readfirstlane(next);
            if (i >= cnt) break;
            bispec_one<N, K, MODE>(item_at(bt, beg + i, n_items), lds0, lds1, bt, spec, n_items, items, group_xy, slot,
                             out_idx, bispec, s_count, acc);
        }
    }
}

__global__ void k_queue_reset(int *queue) {
    if (threadIdx.x < 8) queue[threadIdx.x] = 0;
}

template <int N, int K, int MODE>
hipError_t launch_bispec_t(const BispecArgs &a, int total, hipStream_t st) {
    if (a.form == 0) {
        hipLaunchKernelGGL((k_bispec<N, K, MODE>), dim3(total), dim3(NT), 0, st, a.bt, a.spectra, a.n_items, total,
                           a.items, a.group_xy, a.slot_v, a.out_idx, a.bispec, a.s_count, a.acc);
        return hipGetLastError();
    }
    if (!a.queue) return hipErrorInvalidValue;
    static int resident[2][3] = {{0, 0, 0}, {0, 0, 0}};   // workgroups per CU, per slot count and mode
    int &per_cu = resident[K == 16 ? 0 : 1][MODE];
    if (per_cu == 0) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void *)k_bispec_queue<N, K, MODE>, NT, 0) != hipSuccess || n < 1)
            n = 1;
        per_cu = n;
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return hipErrorInvalidValue;
    const int grid = std::max(8, std::min(total, per_cu * cus) / 8 * 8);
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, st, a.queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_bispec_queue<N, K, MODE>), dim3(grid), dim3(NT), 0, st, a.bt, a.spectra, a.n_items, total,
                       a.items, a.group_xy, a.slot_v, a.out_idx, a.bispec, a.s_count, a.acc, a.queue);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_bispec(const BispecArgs &a, hipStream_t st) {
    const int64_t total64 = (int64_t)a.bt.patches * a.n_items;
    if (total64 == 0) return hipSuccess;
    if (total64 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    const int total = (int)total64;
    if (a.acc.mode < 0 || a.acc.mode > 2) return hipErrorInvalidValue;
    // photon-noise terms in the streaming form: the last group only
    if (a.acc.mode == 1 && a.acc.noise_c) return hipErrorInvalidValue;
    if (a.acc.noise_c && !a.acc.noise_t) return hipErrorInvalidValue;
    if (a.acc.mode != 0) {
        if (a.slots == 16) return a.N == 128 ? launch_bispec_t<128, 16, 1>(a, total, st) : launch_bispec_t<64, 16, 1>(a, total, st);
        if (a.slots == 24) return a.N == 128 ? launch_bispec_t<128, 24, 1>(a, total, st) : launch_bispec_t<64, 24, 1>(a, total, st);
        return hipErrorInvalidValue;
    }
    if (a.acc.noise_c) {
        if (!a.acc.noise_t) return hipErrorInvalidValue;
        if (a.slots == 16) return a.N == 128 ? launch_bispec_t<128, 16, 2>(a, total, st) : launch_bispec_t<64, 16, 2>(a, total, st);
        if (a.slots == 24) return a.N == 128 ? launch_bispec_t<128, 24, 2>(a, total, st) : launch_bispec_t<64, 24, 2>(a, total, st);
        return hipErrorInvalidValue;
    }
    if (a.slots == 16) return a.N == 128 ? launch_bispec_t<128, 16, 0>(a, total, st) : launch_bispec_t<64, 16, 0>(a, total, st);
    if (a.slots == 24) return a.N == 128 ? launch_bispec_t<128, 24, 0>(a, total, st) : launch_bispec_t<64, 24, 0>(a, total, st);
    return hipErrorInvalidValue;
}

}  // namespace nvsm
