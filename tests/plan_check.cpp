// Host check of the work plans the kernels index with (no GPU): for each
// (N, u_cut, R, slots per wave) given on the command line as N:uc:R:K it
// verifies that
//  * every LDS offset a bispectrum lane forms lies inside its item's staged
//    region, every region fits the LDS buffer, and every staged spectrum
//    offset lies inside a stored record;
//  * every sample (w, v) of S is computed exactly once, at the output index
//    of that very (w, v);
//  * the least-squares rounds are consistent: every target of a round's
//    samples is an inner entry or lies in the round's live window, the
//    window fits the accumulator ring, and the flushed prefixes grow to |W|.
// Prints one line per case ending in "bad=<count>"; exit status 0.
#include "plan.hpp"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

using namespace nvsm;

// Stored rows below 0 in a frame's spectrum record (rows -16 .. N/2-1), as
// the kernels store them.
constexpr int SPEC_NEG_ROWS_HOST = 16;

static long check_bispectrum(const HostPlan &pl, int N, int K) {
    long bad = 0;
    const int HALF = N / 2;
    std::vector<int> hit(pl.s_count, 0);
    std::vector<int32_t> wv;
    enumerate_S(pl.uc, pl.R, &wv);
    for (int g = 0; g < pl.n_items; ++g) {
        const int *it = &pl.items[(size_t)g * BS_ITEM_INTS];
        const int gi = it[0], rx0 = it[1], ry0 = it[2], rw = it[3], rh = it[4], npts = it[5], pitch = it[6];
        if (gi < 0 || gi >= pl.n_groups) { ++bad; continue; }
        if (npts > bs_max_region(K) || npts != rw * rh || pitch != rw || (pitch & 1) || (rx0 & 1)) ++bad;
        // staged rows: region rows map to stored rows -16 .. N/2-1 (clamped above)
        if (ry0 < -SPEC_NEG_ROWS_HOST) ++bad;
        for (int wave = 0; wave < BS_WAVES; ++wave) {
            const int ns = it[8 + wave];
            if (ns % 4 || ns > K || ns < 0) ++bad;
            for (int k = 0; k < K; ++k) {
                const size_t sidx = ((size_t)(g * BS_WAVES + wave) * K + k);
                const int roff = pl.slot_v[sidx * 2], so = pl.slot_v[sidx * 2 + 1];
                if (so < 0 || so >= (HALF + SPEC_NEG_ROWS_HOST) * N) { ++bad; continue; }
                const int vy = so / N - SPEC_NEG_ROWS_HOST;
                int vx = so % N;
                if (vx > HALF) vx -= N;
                if (roff != vy * pitch + vx) ++bad;
                for (int lane = 0; lane < BS_LANES; ++lane) {
                    const int wx = pl.group_xy[((size_t)gi * BS_LANES + lane) * 2];
                    const int wy = pl.group_xy[((size_t)gi * BS_LANES + lane) * 2 + 1];
                    if (wy < 0 || wy >= HALF) ++bad;
                    const int a = (wy - ry0) * pitch + (wx - rx0) - roff;   // the kernel's LDS offset
                    if (a < 0 || a >= npts) ++bad;
                    const int o = pl.out_idx[sidx * 64 + lane];
                    if (o >= pl.s_count || (k >= ns && o >= 0)) ++bad;
                    if (o >= 0) {
                        ++hit[o];
                        if (wv[4 * (size_t)o] != wx || wv[4 * (size_t)o + 1] != wy || wv[4 * (size_t)o + 2] != vx ||
                            wv[4 * (size_t)o + 3] != vy)
                            ++bad;
                    }
                }
            }
        }
    }
    for (int64_t i = 0; i < pl.s_count; ++i)
        if (hit[i] != 1) ++bad;
    return bad;
}

static long check_lsq_rounds(const HostPlan &pl) {
    long bad = 0;
    const int nW = (int)pl.W.size() / 2, rounds = (nW + LSQ_ROUND - 1) / LSQ_ROUND;
    const int ring = LSQ_ACC - pl.n_inner;
    if ((int)pl.lsq_fin.size() != rounds + 1 || pl.lsq_fin[0] != pl.n_inner || pl.lsq_fin[rounds] != nW) return 1;
    if (pl.n_inner + pl.lsq_span > LSQ_ACC || 2 * ring <= nW) ++bad;
    for (int r = 0; r < rounds; ++r) {
        const int hi = std::min(nW, (r + 1) * LSQ_ROUND);
        auto live = [&](int x) { return x < pl.n_inner || (x >= pl.lsq_fin[r] && x < hi); };
        for (int w = r * LSQ_ROUND; w < hi; ++w) {
            if (!live(w)) ++bad;
            for (int32_t t = pl.woff[w]; t < pl.woff[w + 1]; ++t) {
                if (!live((int)((pl.phase_code[t] >> 16) & 0x7fffu))) ++bad;
                if (!live((int)(pl.phase_code[t] & 0x7fffu))) ++bad;
            }
        }
        if (hi - pl.lsq_fin[r] > ring) ++bad;
        if (pl.lsq_fin[r + 1] < pl.lsq_fin[r]) ++bad;
    }
    return bad;
}

int main(int argc, char **argv) {
    for (int i = 1; i < argc; ++i) {
        int N = 0, uc = 0, R = 0, K = 0;
        if (std::sscanf(argv[i], "%d:%d:%d:%d", &N, &uc, &R, &K) != 4) {
            std::printf("%s: bad argument bad=1\n", argv[i]);
            continue;
        }
        HostPlan pl;
        std::string err;
        if (!build_plan(N, uc, R, K, &pl, &err)) {
            std::printf("N=%d uc=%d R=%d K=%d: plan failed (%s) bad=1\n", N, uc, R, K, err.c_str());
            continue;
        }
        const long b1 = check_bispectrum(pl, N, K), b2 = check_lsq_rounds(pl);
        std::printf("N=%d uc=%d R=%d K=%d items=%d |S|=%lld bispectrum bad=%ld rounds bad=%ld bad=%ld\n", N, uc, R,
                    K, pl.n_items, (long long)pl.s_count, b1, b2, b1 + b2);
    }
    return 0;
}
