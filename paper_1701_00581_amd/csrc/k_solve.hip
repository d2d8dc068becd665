// Fourier modulus (Eq. 1) and phase (speckle-masking recursion), FP64.
//
// One workgroup per patch.  Frequencies are visited shell by shell (|w|^2
// ascending); every w of a shell reads only strictly shorter frequencies,
// so a shell's w are independent.  The planner joins consecutive shells
// into groups while no w of a group reads another w of it (1161 shells
// make 996 groups at N = 128, |w| <= 63, R = 12), and cuts each group
// into units of at most 8 w; in a unit wave j takes w
// number j, its lanes split that w's bispectrum samples, and a wave
// reduction (DPP) gives
//   z(w) = sum_v e(w - v) e(v) conj B(w, v),  e(w) = z / |z|.
// The workgroup waits at a barrier only after the last unit of a group.
// Since |v| <= R, a group only reads phasors with |x| <= R or
// |x| >= |w| - R: those stay in LDS (the inner disk, plus a ring for the
// annulus), which keeps the workgroup small enough for three per CU.  The
// sample codes hold the LDS slot of each phasor for the sample's group
// (computed on the host), so a lookup is a plain LDS read.  Each phasor is
// written to the output as soon as it is known.  The samples of the next
// DEPTH - 1 units are loaded into registers while the current unit is
// computed: a unit's own work is shorter than a load from HBM, so with a
// single unit in flight the chain of groups waited on memory latency (one w
// per wave and unit keeps a register set small enough for several in flight
// at six waves per SIMD).
#include "device_common.hpp"
#include "kernels.hpp"
#include "plan.hpp"

namespace nvsm {

namespace {

constexpr int NT = 512;
constexpr int NWAVE = NT / 64;
// units of samples in registers (DEPTH - 1 loading).  Two units ahead
// cover the memory latency (a unit takes about 1.7 us); with 4 samples per
// lane the registers a deeper ring would hold go to the unit's phasor
// gathers, which are all issued before its arithmetic (80 VGPRs at 6 waves
// per SIMD; 128 at 4 with 8 samples per lane)
template <int TPL> constexpr int depth_of() { return TPL <= 2 ? 5 : 3; }
static_assert(NWAVE == SOLVE_WAVES, "one w per wave and unit");

__device__ __forceinline__ double2 unit_or_one(double2 z) {
    const double m = sqrt(z.x * z.x + z.y * z.y);
    if (m == 0.0) return make_double2(1.0, 0.0);
    return make_double2(z.x / m, z.y / m);
}

// LDS phasor window: inner entries + ring entries (two sizes)
template <int BIG> struct Win;
template <> struct Win<0> { static constexpr int INNER = 416, RING = 2560; };
template <> struct Win<1> { static constexpr int INNER = 512, RING = 3072; };

// Sum over the 64 lanes with DPP row operations; the total lands in lane 63.
// Every step reads a valid source lane for lane 63 (and bound_ctrl gives 0
// to lanes without one), so no lane needs an initial value.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const int lo = __builtin_amdgcn_mov_dpp((int)__double2loint(v), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)__double2hiint(v), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_total_lane63(double v) {
    v += dpp_d<0xb1>(v);     // quad_perm [1,0,3,2]
    v += dpp_d<0x4e>(v);     // quad_perm [2,3,0,1]
    v += dpp_d<0x141>(v);    // row_half_mirror
    v += dpp_d<0x140>(v);    // row_mirror: every lane holds its row sum
    v += dpp_d<0x142>(v);    // row_bcast:15: row 3 gets rows 2 + 3, row 1 rows 0 + 1
    v += dpp_d<0x143>(v);    // row_bcast:31: row 3 gets the total
    return v;
}

// Samples of one unit for this lane: lane l takes samples l, l + 64, ...
// of the wave's w (w and bar are wave-uniform).
template <int TPL>
struct UnitRegs {
    int w, bar, slot;
    unsigned code[TPL];
    float2 b[TPL];
};

template <int N, int TPL, int BIG>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(TPL <= 4 ? 6 : 2))) void k_solve(int nW, int n_units, const int *__restrict__ units,
                                              int zero_slot, const unsigned *__restrict__ code,
                                              const int *__restrict__ Wxy, const float *__restrict__ power,
                                              const float *__restrict__ mean_spec,
                                              const float2 *__restrict__ bispec, int64_t s_count,
                                              const BurstTable bt, double floor_, int noise_bias,
                                              double *__restrict__ amp, double2 *__restrict__ phasor) {
    __shared__ double2 e[Win<BIG>::INNER + Win<BIG>::RING + 1];   // + the zero phasor
    __shared__ double red[NWAVE];
    const int patch = blockIdx.x;
    const double *stf = bt.b[burst_of(bt, patch, [](const BurstDesc &d) { return (int64_t)d.patch0; })].stf;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const float *P = power + (size_t)patch * N * N;
    double2 *ph_out = phasor + (size_t)patch * nW;

    // noise level: mean power where |u| > N/2 + 2 (signed u in [-N/2, N/2))
    double nb = 0.0;
    if (noise_bias) {
        double acc = 0.0;
        int cnt = 0;
        const double lim = (N / 2 + 2.0) * (N / 2 + 2.0);
        // (every value is loaded, so that the loads of the unrolled passes go
        // out together; the sum runs in the same order)
        static_assert(N * N % NT == 0, "whole passes");
#pragma unroll 8
        for (int j = tid; j < N * N; j += NT) {
            int ux = j % N, uy = j / N;
            ux = ux >= N / 2 ? ux - N : ux;
            uy = uy >= N / 2 ? uy - N : uy;
            const double pj = (double)P[j];
            if ((double)(ux * ux + uy * uy) > lim) { acc += pj; ++cnt; }
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
    // modulus, Eq. 1 (loads unconditional, so that unrolled passes overlap)
#pragma unroll 4
    for (int i = tid; i < nW; i += NT) {
        const int wx = Wxy[2 * i], wy = Wxy[2 * i + 1];
        const int j = (wy & (N - 1)) * N + (wx & (N - 1));
        const double s = stf[j];
        const double num = (double)P[j] - nb;
        double a = 0.0;
        if (s >= floor_) a = sqrt((num > 0.0 ? num : 0.0) / s);
        amp[(size_t)patch * nW + i] = a;
    }
    // seeds (1,0) and (0,1) are W[0] and W[1], inner entries
    if (tid == 0) {
        const float *m = mean_spec + (size_t)patch * 4;
        const double2 e0 = unit_or_one(make_double2((double)m[0], (double)m[1]));
        const double2 e1 = unit_or_one(make_double2((double)m[2], (double)m[3]));
        e[0] = e0;
        e[1] = e1;
        e[zero_slot] = make_double2(0.0, 0.0);
        ph_out[0] = e0;
        ph_out[1] = e1;
    }

    // B of this patch through a buffer resource: a read past the patch's
    // samples returns zero (those lanes' codes are padding anyway)
    const __amdgpu_buffer_rsrc_t brsrc =
        __builtin_amdgcn_make_buffer_rsrc((void *)(bispec + (size_t)patch * s_count), (short)0,
                                          (int)(s_count * (int64_t)sizeof(float2)), 0x00020000);
    constexpr int DEPTH = depth_of<TPL>();
    constexpr int PAD = 64 * TPL;
    // A unit's table entry (this wave's w, first sample, count and barrier
    // flag, LDS slot of the phasor) is read one unit before its samples are
    // requested, so neither the sample loads nor the phasor's store wait on
    // a table read.
    auto entry = [&](int u) __attribute__((always_inline)) {
        const int *t = units + ((size_t)u * NWAVE + wave) * 4;
        return make_int4(t[0], t[1], t[2], t[3]);
    };
    // The code block of the wave's w holds PAD codes (padding: two reads of
    // the zero phasor), so every lane reads TPL codes and TPL samples of B
    // without a bounds test; a padding sample adds zero whatever B it read.
    auto load = [&](const int4 t, UnitRegs<TPL> &r) __attribute__((always_inline)) {
        r.w = t.x;
        r.bar = t.z >> 16;
        r.slot = t.w;
        const unsigned *cw = code + (size_t)max(t.x, 0) * PAD;
        const int b0 = (t.y + lane) * (int)sizeof(float2);
#pragma unroll
        for (int i = 0; i < TPL; ++i) {
            r.code[i] = cw[lane + 64 * i];
            // the whole byte offset in the lane's register (none in the
            // instruction's offset field), so the range test covers all of it
            int off;
            asm("v_add_u32 %0, %2, %1" : "=v"(off) : "v"(b0), "i"(64 * (int)sizeof(float2) * i));
            const auto v = __builtin_amdgcn_raw_buffer_load_b64(brsrc, off, 0, 0);
            r.b[i] = make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
        }
    };
    // Branch-free over the samples, so that the compiler knows how many
    // loads are in flight at every use and waits only for the unit's own.
    // A code holds the LDS slots of e(w - v) (bits 16..30) and e(v) (bits
    // 0..14), each with a conjugation flag above it (bits 31 and 15).
    auto solve = [&](const UnitRegs<TPL> &r) __attribute__((always_inline)) {
        if (r.w < 0) return;                      // no w of this unit in this wave
        double zx = 0.0, zy = 0.0;
        // every gather of the unit first, so that their LDS latency is paid
        // once (the scheduler otherwise waited for each sample's pair in turn)
        double2 ga[TPL], gb[TPL];
#pragma unroll
        for (int i = 0; i < TPL; ++i) {
            ga[i] = e[(r.code[i] >> 16) & 0x7fffu];
            gb[i] = e[r.code[i] & 0x7fffu];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < TPL; ++i) {
            const unsigned cd = r.code[i];
            double2 ea = ga[i];
            double2 eb = gb[i];
            // conjugation: the flag bit moved onto the sign of the imaginary part
            ea.y = __longlong_as_double(__double_as_longlong(ea.y) ^ ((long long)(cd & 0x80000000u) << 32));
            eb.y = __longlong_as_double(__double_as_longlong(eb.y) ^ ((long long)((cd << 16) & 0x80000000u) << 32));
            const double px = fma(ea.x, eb.x, -ea.y * eb.y);
            const double py = fma(ea.x, eb.y, ea.y * eb.x);
            const double bx = (double)r.b[i].x, by = (double)r.b[i].y;
            // z += (px + i py) * conj(bx + i by)
            zx = fma(px, bx, fma(py, by, zx));
            zy = fma(py, bx, fma(-px, by, zy));
        }
        const double tx = wave_total_lane63(zx);
        const double ty = wave_total_lane63(zy);
        if (lane == 63) {
            const double n = tx * tx + ty * ty;
            double2 v = make_double2(1.0, 0.0);
            if (n > 0.0) {
                const double rn = rsqrt(n);
                v = make_double2(tx * rn, ty * rn);
            }
            e[r.slot] = v;
            ph_out[r.w] = v;
        }
    };

    __syncthreads();
    // units in order; the samples of unit u + DEPTH - 1 are requested while
    // unit u is solved (a ring of DEPTH register sets).  Every step requests
    // one unit (past the end: the last unit again, never solved), so the
    // number of loads in flight is the same at every step.
    UnitRegs<TPL> buf[DEPTH];
#pragma unroll
    for (int d = 0; d < DEPTH - 1; ++d) load(entry(min(d, n_units - 1)), buf[d]);
    int4 next = entry(min(DEPTH - 1, n_units - 1));
    for (int u0 = 0; u0 < n_units; u0 += DEPTH) {
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) {
            const int u = u0 + d;
            load(next, buf[(d + DEPTH - 1) % DEPTH]);
            next = entry(min(u + DEPTH, n_units - 1));
            if (u < n_units) {
                solve(buf[d]);
                if (buf[d].bar) __syncthreads();
            }
        }
    }
}

// Least-squares refinement of the phasors of one patch per workgroup (FP64).
// The phasor table of the patch sits in LDS.  Each step computes, for every
// u but the two seeds, g(u) = the sum over the samples holding u of the
// derivative of the closure agreement by conj e(u):
//   u as the sample's w:   e(w - v) e(v) conj B
//   u as the side w - v:   conj e(v) e(w) B
//   u as the side v:       conj e(w - v) e(w) B
// conjugated where the sample holds -u, and the new phasor
// e'(u) = unit(unit(g) + e(u)), all from the previous step's table (Jacobi).
// The samples are read once per step in storage order (one w per wave, its
// samples over the lanes), so B streams contiguously; each contribution is
// added to the accumulator of its target in LDS.  W is ordered by |w|^2
// and both sides of a sample are shorter than its w (|w - v| >= |w| - R),
// so as the segments advance, the entries below some prefix are targeted by
// no later segment: the segments are taken in rounds of LSQ_ROUND, and
// after each round the entries that have just become final (a prefix of W
// beyond the inner disk, from the plan's table lsq_fin) are turned into new
// phasors and their accumulators cleared.  So accumulators are needed only
// for the inner disk (|u| <= R, the sides v of every segment, final at the
// end) and a ring over the live annulus, which fit in LDS beside the table.
// The adds are 64-bit fixed point (scale 2^60 / sum |Re B| + |Im B| of the
// patch, which bounds every |g| below 2^62): integer sums do not depend on
// the order of the adds, so the result is reproducible bit for bit.  Thread
// i keeps e'(u) for u = i + 1024 m in registers until the step ends; then
// the table is rewritten between two barriers.
constexpr int LSQ_MAXW = 6240;
constexpr int LSQ_NT = 1024;                 // 16 waves: the one workgroup a CU holds hides latency
constexpr int LSQ_NWAVE = LSQ_NT / 64;
constexpr int LSQ_SLOTS = (LSQ_MAXW + LSQ_NT - 1) / LSQ_NT;
constexpr int LSQ_UNROLL = 2;
static_assert(LSQ_ROUND % LSQ_NWAVE == 0, "a round gives every wave the same number of segments");

__global__ __launch_bounds__(LSQ_NT) void k_lsq(int nW, int n_inner, int iters, const int *__restrict__ woff,
                                            const unsigned *__restrict__ code, const int *__restrict__ fin,
                                            const float2 *__restrict__ bispec, int64_t s_count,
                                            double2 *__restrict__ phasor) {
    __shared__ double2 e[LSQ_MAXW];
    __shared__ unsigned long long acc[2 * LSQ_ACC];
    __shared__ double red[LSQ_NWAVE];
    const int patch = blockIdx.x;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    double2 *ph = phasor + (size_t)patch * nW;
    const float2 *B = bispec + (size_t)patch * s_count;
    for (int i = tid; i < nW; i += LSQ_NT) e[i] = ph[i];
    // fixed-point scale from sum |Re B| + |Im B| (fixed summation order)
    // (eight loads in flight per thread: clamped past the end, and weighted 0)
    double s1 = 0.0;
    for (int64_t t0 = tid; t0 < s_count; t0 += 8 * LSQ_NT) {
        float2 v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = B[min(t0 + (int64_t)k * LSQ_NT, s_count - 1)];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (t0 + (int64_t)k * LSQ_NT < s_count) s1 += fabs((double)v[k].x) + fabs((double)v[k].y);
    }
    s1 = wave_sum_d(s1);
    if (lane == 0) red[wave] = s1;
    __syncthreads();
    s1 = 0.0;
#pragma unroll
    for (int k = 0; k < LSQ_NWAVE; ++k) s1 += red[k];
    if (!(s1 > 0.0) || !isfinite(s1)) return;          // no usable samples: the phasors stay
    const double scale = 0x1p60 / s1, inv_scale = s1 * 0x1p-60;
    const int ring = LSQ_ACC - n_inner;                 // >= the plan's live span (checked on the host)
    // accumulator of entry x: the inner disk first, then the ring
    auto slot = [&](unsigned x) __attribute__((always_inline)) {
        if ((int)x < n_inner) return x;
        int q = (int)x - n_inner;
        if (q >= ring) q -= ring;                       // x - n_inner < |W| < 2 ring
        return (unsigned)(n_inner + q);
    };
    auto get = [&](unsigned c) __attribute__((always_inline)) {     // e of a code (index | conj << 15)
        double2 v = e[c & 0x7fffu];
        if (c & 0x8000u) v.y = -v.y;
        return v;
    };
    auto add = [&](unsigned k, double x, double y) __attribute__((always_inline)) {
        atomicAdd(&acc[2 * k], (unsigned long long)__double2ll_rn(x * scale));
        atomicAdd(&acc[2 * k + 1], (unsigned long long)__double2ll_rn(y * scale));
    };
    const int rounds = (nW + LSQ_ROUND - 1) / LSQ_ROUND;
    for (int it = 0; it < iters; ++it) {
        double2 res[LSQ_SLOTS];
        for (int i = tid; i < 2 * LSQ_ACC; i += LSQ_NT) acc[i] = 0ull;
        __syncthreads();
        for (int r = 0; r < rounds; ++r) {
            // This wave's segments of the round, w = r LSQ_ROUND + wave, + LSQ_NWAVE, ...,
            // taken in chunks of 64 LSQ_UNROLL samples.  The loads of the next chunk
            // (of this segment or the next) are issued before the current chunk is
            // computed, so their latency runs under its arithmetic.  Every lane loads
            // (past a segment's end: its last sample, or sample 0 of an empty one,
            // unused), so the compiler knows how many loads are in flight.
            const int wend = min(nW, (r + 1) * LSQ_ROUND);
            int w = r * LSQ_ROUND + wave;
            if (w < wend) {
                unsigned cd[2][LSQ_UNROLL];
                float2 bb[2][LSQ_UNROLL];
                auto load = [&](int buf, int tb, int t1) __attribute__((always_inline)) {
#pragma unroll
                    for (int k = 0; k < LSQ_UNROLL; ++k) {
                        const int t = max(min(tb + 64 * k + lane, t1 - 1), 0);
                        cd[buf][k] = code[t];
                        bb[buf][k] = B[t];
                    }
                };
                int t1 = woff[w + 1], tb = woff[w];
                load(0, tb, t1);
                double gx = 0.0, gy = 0.0;
                double2 cw = e[w];
                auto step = [&](int cur) __attribute__((always_inline)) {
                    // the next chunk: the rest of this segment, else the next segment
                    int nw = w, ntb = tb + 64 * LSQ_UNROLL, nt1 = t1;
                    const bool seg_end = ntb >= t1;
                    if (seg_end) {
                        nw = w + LSQ_NWAVE;
                        if (nw < wend) { ntb = woff[nw]; nt1 = woff[nw + 1]; }
                    }
                    const bool more = nw < wend;
                    // (unconditional: past the round's last chunk the indices clamp
                    // to a sample of this segment, unused)
                    load(cur ^ 1, ntb, nt1);
#pragma unroll
                    for (int k = 0; k < LSQ_UNROLL; ++k) {
                        if (tb + 64 * k + lane >= t1) continue;
                        const unsigned c = cd[cur][k];
                        const double2 a = get(c >> 16), b = get(c & 0xffffu);
                        const double bx = (double)bb[cur][k].x, by = (double)bb[cur][k].y;
                        // own: (a b) conj(B)
                        const double px = a.x * b.x - a.y * b.y, py = a.x * b.y + a.y * b.x;
                        gx += px * bx + py * by;
                        gy += py * bx - px * by;
                        {   // side w - v: conj(b) e(w) B
                            const double qx = b.x * cw.x + b.y * cw.y, qy = b.x * cw.y - b.y * cw.x;
                            const double ry = qx * by + qy * bx;
                            add(slot((c >> 16) & 0x7fffu), qx * bx - qy * by, (c >> 31) ? -ry : ry);
                        }
                        {   // side v: conj(a) e(w) B
                            const double qx = a.x * cw.x + a.y * cw.y, qy = a.x * cw.y - a.y * cw.x;
                            const double ry = qx * by + qy * bx;
                            add(slot(c & 0x7fffu), qx * bx - qy * by, (c & 0x8000u) ? -ry : ry);
                        }
                    }
                    if (seg_end) {
                        gx = wave_sum_d(gx);
                        gy = wave_sum_d(gy);
                        if (lane == 0) add(slot((unsigned)w), gx, gy);
                        gx = 0.0;
                        gy = 0.0;
                        if (more) cw = e[nw];
                    }
                    w = nw;
                    tb = ntb;
                    t1 = nt1;
                    return more;
                };
                // two chunks per pass, so that the register sets alternate statically
                while (step(0) && step(1)) {
                }
            }
            __syncthreads();
            // entries no later round targets: new phasors, accumulators cleared
            // for the ring entries that will take their slots
            const int f0 = fin[r], f1 = fin[r + 1];
            const bool last = r + 1 == rounds;
#pragma unroll
            for (int j = 0; j < LSQ_SLOTS; ++j) {
                const int u = tid + LSQ_NT * j;
                if (u >= 2 && u < nW && ((u >= f0 && u < f1) || (last && u < n_inner))) {
                    const unsigned k = slot((unsigned)u);
                    const double gx = (double)(long long)acc[2 * k] * inv_scale;
                    const double gy = (double)(long long)acc[2 * k + 1] * inv_scale;
                    acc[2 * k] = 0ull;
                    acc[2 * k + 1] = 0ull;
                    const double2 old = e[u];
                    double2 nw = old;
                    const double m = sqrt(gx * gx + gy * gy);
                    if (m > 0.0) {
                        const double sx = gx / m + old.x, sy = gy / m + old.y;
                        const double rr = sqrt(sx * sx + sy * sy);
                        if (rr > 0.0) nw = make_double2(sx / rr, sy / rr);
                    }
                    res[j] = nw;
                }
            }
            __syncthreads();                               // cleared before the next round adds
        }
#pragma unroll
        for (int j = 0; j < LSQ_SLOTS; ++j) {
            const int u = tid + LSQ_NT * j;
            if (u >= 2 && u < nW) {
                e[u] = res[j];
                if (it + 1 == iters) ph[u] = res[j];
            }
        }
        __syncthreads();
    }
}

template <int N, int TPL, int BIG>
hipError_t launch_solve_t(const SolveArgs &a, hipStream_t st) {
    hipLaunchKernelGGL((k_solve<N, TPL, BIG>), dim3(a.bt.patches), dim3(NT), 0, st, a.nW, a.n_units, a.units,
                       a.zero_slot, a.code, a.Wxy, a.power, a.mean_spec, a.bispec,
                       a.s_count, a.bt, a.floor, a.noise_bias, a.amp, a.phasor);
    return hipGetLastError();
}

template <int N, int BIG>
hipError_t launch_solve_n(const SolveArgs &a, hipStream_t st) {
    switch (solve_samples_per_lane(a.max_sw)) {
    case 2: return launch_solve_t<N, 2, BIG>(a, st);
    case 4: return launch_solve_t<N, 4, BIG>(a, st);
    default: return launch_solve_t<N, 8, BIG>(a, st);
    }
}

}  // namespace

hipError_t launch_lsq(const SolveArgs &a, hipStream_t st) {
    if (a.nW > LSQ_MAXW || a.nW < 2 || a.lsq_iters < 1 || !a.lsq_fin) return hipErrorInvalidValue;
    if (a.n_inner < 2 || a.n_inner > LSQ_ACC / 2 || 2 * (LSQ_ACC - a.n_inner) <= a.nW) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_lsq, dim3(a.bt.patches), dim3(LSQ_NT), 0, st, a.nW, a.n_inner, a.lsq_iters, a.woff, a.wcode,
                       a.lsq_fin, a.bispec, a.s_count, a.phasor);
    return hipGetLastError();
}

hipError_t launch_solve(const SolveArgs &a, hipStream_t st) {
    if (a.bt.patches == 0) return hipSuccess;
    if (a.phase_method == 1) {
        hipError_t e = launch_solve(SolveArgs(a, 0), st);
        return e != hipSuccess ? e : launch_lsq(a, st);
    }
    if (a.max_sw > SOLVE_MAX_SAMPLES || a.zero_slot != a.n_inner + a.ring) return hipErrorInvalidValue;
    if (a.s_count * (int64_t)sizeof(float2) > INT32_MAX) return hipErrorInvalidValue;   // buffer range of B
    const bool small = a.n_inner <= Win<0>::INNER && a.ring <= Win<0>::RING;
    if (!small && (a.n_inner > Win<1>::INNER || a.ring > Win<1>::RING)) return hipErrorInvalidValue;
    if (a.N == 128) return small ? launch_solve_n<128, 0>(a, st) : launch_solve_n<128, 1>(a, st);
    return small ? launch_solve_n<64, 0>(a, st) : launch_solve_n<64, 1>(a, st);
}

}  // namespace nvsm
