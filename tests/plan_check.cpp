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
//    window fits the accumulator ring, and the flushed prefixes grow to |W|;
//  * the phase-solve units cover W in order, and each w's padded code block
//    holds its own sample codes followed by reads of the zero phasor's slot.
// Prints one line per case ending in "bad=<count>"; exit status 0.
// A case written shells:N:uc:R:K re-plans the phase solve with one group
// per shell; merge:N:uc:R:K joins the first two groups after the seeds,
// whose second reads the first, so its check must report a bad count.
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
            if (ns % 4 || ns > K || ns < 4) ++bad;
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

// Phase-solve units: groups are runs of whole shells; every w of groups 1..
// exactly once, in storage order, with its S range; at most SOLVE_WAVES w
// per unit, all of one group; the barrier flag set exactly on each group's
// last unit; and every sample's sides come from strictly earlier groups (so
// the units of a group are independent).
static long check_solve_units(const HostPlan &pl) {
    long bad = 0;
    const int nW = (int)pl.W.size() / 2, ngroup = (int)pl.group_wb.size() - 1;
    if ((int)pl.solve_units.size() != pl.n_units * SOLVE_WAVES * 4) return 1;
    // groups are runs of whole shells, the first of them the seed shell
    if (ngroup < 1 || pl.group_wb[0] != 0 || pl.group_wb[ngroup] != nW) return 1;
    if (ngroup > 1 && pl.group_wb[1] != pl.shell_wb[1]) ++bad;
    for (int g = 1; g <= ngroup; ++g) {
        if (pl.group_wb[g] <= pl.group_wb[g - 1]) return bad + 1;
        if (!std::binary_search(pl.shell_wb.begin(), pl.shell_wb.end(), pl.group_wb[g])) ++bad;
    }
    std::vector<int> group_of(nW);
    for (int g = 0; g < ngroup; ++g)
        for (int w = pl.group_wb[g]; w < pl.group_wb[g + 1]; ++w) group_of[w] = g;
    int expect = ngroup > 1 ? pl.group_wb[1] : nW;
    for (int u = 0; u < pl.n_units; ++u) {
        const int32_t *t = &pl.solve_units[(size_t)u * SOLVE_WAVES * 4];
        const int g = group_of[t[0]];
        const int flag = t[2] >> 16;
        for (int j = 0; j < SOLVE_WAVES; ++j) {
            const int w = t[4 * j], o = t[4 * j + 1], c = t[4 * j + 2] & 0xffff, last = t[4 * j + 2] >> 16;
            if (last != flag) ++bad;
            if (w < 0) {
                if (o != 0 || c != 0) ++bad;
                continue;
            }
            if (w != expect || group_of[w] != g) ++bad;
            ++expect;
            if (o != pl.woff[w] || c != pl.woff[w + 1] - pl.woff[w] || t[4 * j + 3] != pl.w_slot[w]) ++bad;
            for (int32_t k = o; k < o + c; ++k) {
                const int ia = (int)((pl.phase_code[k] >> 16) & 0x7fffu), ib = (int)(pl.phase_code[k] & 0x7fffu);
                if (group_of[ia] >= g || group_of[ib] >= g) ++bad;
            }
        }
        const bool end = expect == pl.group_wb[g + 1];
        if ((flag != 0) != end) ++bad;
    }
    if (expect != nW) ++bad;
    // the phasor window: every sample reads each side at the slot where that
    // side's phasor was written (w_slot), and the ring entries live while a
    // group is solved (from the lowest one its samples read to its own last
    // w) hold distinct slots, so none was overwritten in between
    for (int g = 1; g < ngroup; ++g) {
        int lo = pl.group_wb[g];
        for (int w = pl.group_wb[g]; w < pl.group_wb[g + 1]; ++w)
            for (int32_t t = pl.woff[w]; t < pl.woff[w + 1]; ++t) {
                const uint32_t c = pl.phase_code[t], sc = pl.phase_slot_code[t];
                const int x[2] = {(int)((c >> 16) & 0x7fffu), (int)(c & 0x7fffu)};
                const int sl[2] = {(int)((sc >> 16) & 0x7fffu), (int)(sc & 0x7fffu)};
                for (int k = 0; k < 2; ++k) {
                    if (sl[k] != pl.w_slot[x[k]]) ++bad;
                    if (x[k] >= pl.n_inner) lo = std::min(lo, x[k]);
                }
            }
        std::vector<int> seen(pl.zero_slot, 0);
        for (int x = 0; x < pl.n_inner; ++x) ++seen[pl.w_slot[x]];
        for (int x = std::max(lo, pl.n_inner); x < pl.group_wb[g + 1]; ++x) ++seen[pl.w_slot[x]];
        for (int v : seen)
            if (v > 1) ++bad;
    }
    // the padded code blocks: w's codes, then reads of the zero slot, which
    // lies past every phasor slot
    if (pl.zero_slot != pl.n_inner + pl.ring_size || pl.zero_slot > 0x7fff) ++bad;
    if (pl.solve_pad != 64 * solve_samples_per_lane(pl.max_sw) || pl.solve_pad < pl.max_sw) return bad + 1;
    if (pl.solve_code.size() != (size_t)nW * pl.solve_pad) return bad + 1;
    const uint32_t zero = ((uint32_t)pl.zero_slot << 16) | (uint32_t)pl.zero_slot;
    for (int w = 0; w < nW; ++w) {
        if (pl.w_slot[w] >= pl.zero_slot) ++bad;
        const int cnt = w < pl.shell_wb[1] ? 0 : pl.woff[w + 1] - pl.woff[w];
        for (int k = 0; k < pl.solve_pad; ++k) {
            const uint32_t c = pl.solve_code[(size_t)w * pl.solve_pad + k];
            if (k < cnt) {
                if (c != pl.phase_slot_code[pl.woff[w] + k]) ++bad;
                if ((int)((c >> 16) & 0x7fffu) >= pl.zero_slot || (int)(c & 0x7fffu) >= pl.zero_slot) ++bad;
            } else if (c != zero) {
                ++bad;
            }
        }
    }
    return bad;
}

int main(int argc, char **argv) {
    for (int i = 1; i < argc; ++i) {
        int N = 0, uc = 0, R = 0, K = 0;
        const std::string arg = argv[i];
        const bool shells = arg.rfind("shells:", 0) == 0, merge = arg.rfind("merge:", 0) == 0;
        const char *spec = argv[i] + (shells ? 7 : merge ? 6 : 0);
        if (std::sscanf(spec, "%d:%d:%d:%d", &N, &uc, &R, &K) != 4) {
            std::printf("%s: bad argument bad=1\n", argv[i]);
            continue;
        }
        HostPlan pl;
        std::string err;
        bool ok = build_plan(N, uc, R, K, &pl, &err);
        if (ok && (shells || merge)) {
            if (shells) pl.group_wb = pl.shell_wb;
            if (merge && pl.group_wb.size() > 3) pl.group_wb.erase(pl.group_wb.begin() + 2);
            ok = plan_phase_solve(&pl, &err);
        }
        if (!ok) {
            std::printf("%s: plan failed (%s) bad=1\n", argv[i], err.c_str());
            continue;
        }
        const long b1 = check_bispectrum(pl, N, K), b2 = check_lsq_rounds(pl), b3 = check_solve_units(pl);
        std::printf("%s items=%d shells=%d groups=%d units=%d ring=%d |S|=%lld bispectrum bad=%ld "
                    "rounds bad=%ld units bad=%ld bad=%ld\n", argv[i], pl.n_items, (int)pl.shell_wb.size() - 1,
                    (int)pl.group_wb.size() - 1, pl.n_units, pl.ring_size, (long long)pl.s_count, b1, b2, b3, b1 + b2 + b3);
    }
    return 0;
}
