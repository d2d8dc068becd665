// Host-side planning for the speckle-masking path (see plan.hpp).
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <unordered_map>

namespace nvsm {

bool make_tiling(int H, int W, int N, int s, Tiling *t) {
    if (N <= 0 || s <= 0 || H < N || W < N) return false;
    auto axis = [&](int L, std::vector<int32_t> *o) {
        int n = (L - N + s - 1) / s + 1;
        o->resize(n);
        for (int k = 0; k < n; ++k) (*o)[k] = std::min(k * s, L - N);
    };
    axis(H, &t->ys);
    axis(W, &t->xs);
    t->ny = (int)t->ys.size();
    t->nx = (int)t->xs.size();
    return true;
}

static inline bool upper_half(int x, int y) { return y > 0 || (y == 0 && x > 0); }

void enumerate_W(int uc, std::vector<int32_t> *w) {
    struct P { int x, y; };
    std::vector<P> pts;
    for (int y = 0; y <= uc; ++y)
        for (int x = -uc; x <= uc; ++x) {
            int r2 = x * x + y * y;
            if (r2 == 0 || r2 > uc * uc || !upper_half(x, y)) continue;
            pts.push_back({x, y});
        }
    std::sort(pts.begin(), pts.end(), [](const P &a, const P &b) {
        int ra = a.x * a.x + a.y * a.y, rb = b.x * b.x + b.y * b.y;
        if (ra != rb) return ra < rb;
        if (a.y != b.y) return a.y < b.y;
        return a.x < b.x;
    });
    w->clear();
    for (auto &p : pts) { w->push_back(p.x); w->push_back(p.y); }
}

// Appends the v of S(w) in (vy, vx) order.
static void samples_of(int wx, int wy, int R, std::vector<int32_t> *v) {
    int n2 = wx * wx + wy * wy;
    for (int vy = -R; vy <= R; ++vy)
        for (int vx = -R; vx <= R; ++vx) {
            int a = vx * vx + vy * vy;
            if (a == 0 || a > R * R || a >= n2) continue;
            int dx = wx - vx, dy = wy - vy, b = dx * dx + dy * dy;
            if (b == 0 || b >= n2) continue;
            v->push_back(vx);
            v->push_back(vy);
        }
}

void enumerate_S(int uc, int R, std::vector<int32_t> *wv) {
    std::vector<int32_t> W;
    enumerate_W(uc, &W);
    wv->clear();
    std::vector<int32_t> v;
    for (size_t i = 0; i < W.size() / 2; ++i) {
        v.clear();
        samples_of(W[2 * i], W[2 * i + 1], R, &v);
        for (size_t j = 0; j < v.size() / 2; ++j) {
            wv->push_back(W[2 * i]);
            wv->push_back(W[2 * i + 1]);
            wv->push_back(v[2 * j]);
            wv->push_back(v[2 * j + 1]);
        }
    }
}

int count_shells(const std::vector<int32_t> &W) {
    int n = 0, last = -1;
    for (size_t i = 0; i < W.size() / 2; ++i) {
        int r2 = W[2 * i] * W[2 * i] + W[2 * i + 1] * W[2 * i + 1];
        if (r2 != last) { ++n; last = r2; }
    }
    return n;
}

bool plan_phase_solve(HostPlan *pl, std::string *err) {
    const int nW = (int)pl->W.size() / 2, R = pl->R;
    // phasor window: inner entries |w| <= R, the rest in a ring; each
    // group's lowest ring entry read comes from its sample codes
    pl->n_inner = 0;
    while (pl->n_inner < nW) {
        const int x = pl->W[2 * pl->n_inner], y = pl->W[2 * pl->n_inner + 1];
        if (x * x + y * y > R * R) break;
        ++pl->n_inner;
    }
    const int ngroup = (int)pl->group_wb.size() - 1;
    std::vector<int32_t> lo(ngroup);
    int span = 1;
    for (int g = 0; g < ngroup; ++g) {
        int l = pl->group_wb[g];
        for (int32_t t = pl->woff[pl->group_wb[g]]; t < pl->woff[pl->group_wb[g + 1]]; ++t) {
            const int ia = (int)((pl->phase_code[t] >> 16) & 0x7fffu), ib = (int)(pl->phase_code[t] & 0x7fffu);
            if (ia >= pl->n_inner) l = std::min(l, ia);
            if (ib >= pl->n_inner) l = std::min(l, ib);
        }
        lo[g] = std::max(l, pl->n_inner);
        span = std::max(span, pl->group_wb[g + 1] - lo[g]);
    }
    pl->ring_size = span;
    pl->group_ring_off.resize(ngroup);
    for (int g = 0; g < ngroup; ++g)
        pl->group_ring_off[g] = (lo[g] - pl->n_inner) / span * span;
    auto slot_of = [&](int i, int ro) {
        if (i < pl->n_inner) return i;
        int q = i - pl->n_inner - ro;
        if (q >= span) q -= span;
        return pl->n_inner + q;
    };
    pl->phase_slot_code.resize(pl->phase_code.size());
    pl->w_slot.resize(nW);
    for (int g = 0; g < ngroup; ++g) {
        const int ro = pl->group_ring_off[g];
        for (int w = pl->group_wb[g]; w < pl->group_wb[g + 1]; ++w) {
            pl->w_slot[w] = slot_of(w, ro);
            for (int32_t t = pl->woff[w]; t < pl->woff[w + 1]; ++t) {
                const uint32_t c = pl->phase_code[t];
                const uint32_t ca = c >> 16, cb = c & 0xffffu;
                const uint32_t sa = (uint32_t)slot_of((int)(ca & 0x7fffu), ro) | (ca & 0x8000u);
                const uint32_t sb = (uint32_t)slot_of((int)(cb & 0x7fffu), ro) | (cb & 0x8000u);
                pl->phase_slot_code[t] = (sa << 16) | sb;
            }
        }
    }
    if (pl->s_count >= (int64_t)1 << 31) { *err = "bispectrum set too large"; return false; }

    // the solve's padded code blocks
    pl->max_sw = 0;
    for (int w = 0; w < nW; ++w) pl->max_sw = std::max(pl->max_sw, pl->woff[w + 1] - pl->woff[w]);
    pl->zero_slot = pl->n_inner + pl->ring_size;
    pl->solve_code.clear();
    pl->solve_pad = 0;
    if (pl->max_sw <= SOLVE_MAX_SAMPLES) {
        pl->solve_pad = 64 * solve_samples_per_lane(pl->max_sw);
        const uint32_t zero = ((uint32_t)pl->zero_slot << 16) | (uint32_t)pl->zero_slot;
        pl->solve_code.assign((size_t)nW * pl->solve_pad, zero);
        for (int w = pl->shell_wb[1]; w < nW; ++w)
            std::copy(pl->phase_slot_code.begin() + pl->woff[w], pl->phase_slot_code.begin() + pl->woff[w + 1],
                      pl->solve_code.begin() + (size_t)w * pl->solve_pad);
    }

    // phase-solve units: groups 1.. cut into runs of SOLVE_WAVES w
    pl->solve_units.clear();
    pl->n_units = 0;
    for (size_t g = 1; g + 1 < pl->group_wb.size(); ++g) {
        const int end = pl->group_wb[g + 1];
        for (int w0 = pl->group_wb[g]; w0 < end; w0 += SOLVE_WAVES) {
            const int last = w0 + SOLVE_WAVES >= end;
            for (int j = 0; j < SOLVE_WAVES; ++j) {
                const int w = w0 + j;
                if (w < end)
                    pl->solve_units.insert(pl->solve_units.end(),
                                           {w, pl->woff[w], (pl->woff[w + 1] - pl->woff[w]) | (last << 16), pl->w_slot[w]});
                else
                    pl->solve_units.insert(pl->solve_units.end(), {-1, 0, last << 16, 0});
            }
            ++pl->n_units;
        }
    }
    return true;
}

bool build_plan(int N, int uc, int R, int K, HostPlan *pl, std::string *err) {
    if (K < 8 || K > BS_MAX_SLOTS || K % 8) { *err = "slots per wave must be 8..32, a multiple of 8"; return false; }
    pl->slots = K;
    if (N != 64 && N != 128) { *err = "patch must be 64 or 128"; return false; }
    if (uc < 2 || uc >= N / 2) { *err = "u_cut must be in [2, N/2)"; return false; }
    if (R < 1 || R > 16 || R >= uc) { *err = "v_radius must be in [1, min(16, u_cut))"; return false; }
    pl->N = N; pl->uc = uc; pl->R = R;
    enumerate_W(uc, &pl->W);
    const int nW = (int)pl->W.size() / 2;
    if (nW >= 0x8000) { *err = "too many frequencies"; return false; }

    // index of each upper-half frequency
    const int side = 2 * uc + 1;
    std::vector<int32_t> widx((size_t)side * side, -1);
    auto at = [&](int x, int y) -> int32_t & { return widx[(size_t)(y + uc) * side + (x + uc)]; };
    for (int i = 0; i < nW; ++i) at(pl->W[2 * i], pl->W[2 * i + 1]) = i;
    auto code = [&](int x, int y) -> uint32_t {
        if (upper_half(x, y)) return (uint32_t)at(x, y);
        return (uint32_t)at(-x, -y) | 0x8000u;
    };

    // S offsets, phase lookup codes, shells; per-w rank maps for the kernel
    pl->woff.assign(nW + 1, 0);
    pl->phase_code.clear();
    pl->shell_wb.clear();
    std::vector<std::vector<int32_t>> Sw(nW);
    int last = -1;
    for (int i = 0; i < nW; ++i) {
        int wx = pl->W[2 * i], wy = pl->W[2 * i + 1];
        int r2 = wx * wx + wy * wy;
        if (r2 != last) { pl->shell_wb.push_back(i); last = r2; }
        samples_of(wx, wy, R, &Sw[i]);
        for (size_t j = 0; j < Sw[i].size() / 2; ++j) {
            int vx = Sw[i][2 * j], vy = Sw[i][2 * j + 1];
            pl->phase_code.push_back((code(wx - vx, wy - vy) << 16) | code(vx, vy));
        }
        pl->woff[i + 1] = pl->woff[i] + (int32_t)(Sw[i].size() / 2);
    }
    pl->shell_wb.push_back(nW);
    pl->s_count = pl->woff[nW];

    // phase-solve groups: a shell joins the group before it when none of
    // its samples reads a w of that group (reads always go to shorter w)
    pl->group_wb.assign(1, 0);
    for (size_t sh = 1; sh + 1 < pl->shell_wb.size(); ++sh) {
        const int g0 = pl->group_wb.back();
        bool reads_group = sh == 1;  // the seed shell is a group of its own
        for (int32_t t = pl->woff[pl->shell_wb[sh]]; t < pl->woff[pl->shell_wb[sh + 1]] && !reads_group; ++t)
            reads_group = (int)((pl->phase_code[t] >> 16) & 0x7fffu) >= g0 || (int)(pl->phase_code[t] & 0x7fffu) >= g0;
        if (reads_group) pl->group_wb.push_back(pl->shell_wb[sh]);
    }
    pl->group_wb.push_back(nW);

    // sample indices are kept in 30 bits by the kernels' tables
    if (pl->s_count >= (int64_t)1 << 30) { *err = "bispectrum set too large"; return false; }

    if (!plan_phase_solve(pl, err)) return false;

    // least-squares rounds: the last segment that targets each entry (as
    // its own w or as a side of one of its samples), then the prefixes of
    // entries that no later round targets
    {
        std::vector<int32_t> last(nW);
        for (int w = 0; w < nW; ++w) {
            last[w] = std::max(last[w], w);
            for (int32_t t = pl->woff[w]; t < pl->woff[w + 1]; ++t) {
                const int ia = (int)((pl->phase_code[t] >> 16) & 0x7fffu), ib = (int)(pl->phase_code[t] & 0x7fffu);
                last[ia] = std::max(last[ia], w);
                last[ib] = std::max(last[ib], w);
            }
        }
        const int rounds = (nW + LSQ_ROUND - 1) / LSQ_ROUND;
        pl->lsq_fin.assign(rounds + 1, nW);
        pl->lsq_span = 0;
        int fin = pl->n_inner;
        for (int r = 0; r < rounds; ++r) {
            while (fin < nW && last[fin] < r * LSQ_ROUND) ++fin;
            pl->lsq_fin[r] = fin;
            pl->lsq_span = std::max(pl->lsq_span, std::min(nW, (r + 1) * LSQ_ROUND) - fin);
        }
    }

    // Bispectrum work.  Lanes of a wave hold a group of up to 64 w that lie
    // close together in angle and radius: for |w| well above R, S(w) is the
    // part of the |v| <= R disk on w's side of a line through the origin
    // normal to w, so w of similar direction share most of their v and the
    // union of their sets (the v slots the wave runs) is little larger
    // than each set.  Groups: radial bands (8 wide up to 16, then about 10
    // wide), each sorted by angle and cut into equal groups of <= 64.
    // Wider bands give narrower angles (fewer idle lanes) but larger staged
    // regions.
    std::vector<int> edges = {0};
    for (int e = 8; e <= 16; e += 8)
        if (e < uc + 1) edges.push_back(e);
    {
        const int lo = edges.back(), parts = std::max(1, (int)std::lround((uc + 1 - lo) / 10.0));
        for (int q = 1; q <= parts; ++q) edges.push_back(lo + (uc + 1 - lo) * q / parts);
    }
    std::vector<std::vector<int>> groups;
    for (size_t bnd = 0; bnd + 1 < edges.size(); ++bnd) {
        const double r0 = edges[bnd], r1 = edges[bnd + 1];
        std::vector<std::pair<double, int>> ws;
        for (int i = 0; i < nW; ++i) {
            const double r = std::sqrt((double)(pl->W[2 * i] * pl->W[2 * i] + pl->W[2 * i + 1] * pl->W[2 * i + 1]));
            if (r >= r0 && r < r1) ws.push_back({std::atan2((double)pl->W[2 * i + 1], (double)pl->W[2 * i]), i});
        }
        if (ws.empty()) continue;
        std::sort(ws.begin(), ws.end());
        const int n = (int)ws.size(), ng = (n + BS_LANES - 1) / BS_LANES;
        for (int q = 0; q < ng; ++q) {
            std::vector<int> gw;
            for (int j = (int)((int64_t)n * q / ng); j < (int)((int64_t)n * (q + 1) / ng); ++j) gw.push_back(ws[j].second);
            groups.push_back(gw);
        }
    }
    pl->n_groups = (int)groups.size();
    pl->group_xy.assign((size_t)pl->n_groups * BS_LANES * 2, 0);
    pl->items.clear();
    pl->slot_v.clear();
    pl->out_idx.clear();
    pl->computed_terms = 0;
    int64_t covered = 0;
    pl->max_region = 0;
    for (int gi = 0; gi < pl->n_groups; ++gi) {
        const std::vector<int> &gset = groups[gi];
        int gx0 = 1 << 20, gx1 = -(1 << 20), gy0 = 1 << 20, gy1 = -(1 << 20);
        std::map<std::pair<int, int>, int> uni;  // (vy, vx) sorted union
        for (int i : gset) {
            const int wx = pl->W[2 * i], wy = pl->W[2 * i + 1];
            gx0 = std::min(gx0, wx); gx1 = std::max(gx1, wx);
            gy0 = std::min(gy0, wy); gy1 = std::max(gy1, wy);
            for (size_t j = 0; j < Sw[i].size() / 2; ++j) uni[{Sw[i][2 * j + 1], Sw[i][2 * j]}] = 1;
        }
        std::vector<std::pair<int, int>> U;  // (vx, vy)
        for (auto &u : uni) U.push_back({u.first.second, u.first.first});
        if (U.empty()) continue;
        // Items: full ones (BS_WAVES chunks of K slots), then one for the
        // rest, whose waves all run ns slots (ns the smallest multiple of 4
        // that holds a quarter of the rest); chunks balanced within an item.
        // Items hold fewer v (in steps of 4 per wave) where the staged
        // region of a full item would not fit the LDS capacity.
        const int nU = (int)U.size();
        struct Item { int u0, m, ns, rx0, ry0, rw, rh; };
        std::vector<Item> gitems;
        int maxw = 0;
        for (int mcap = BS_WAVES * K; mcap > 0; mcap -= 4 * BS_WAVES) {
            gitems.clear();
            maxw = 0;
            int maxh = 0;
            for (int u0 = 0; u0 < nU; u0 += mcap) {
                const int m = std::min(nU - u0, mcap);
                const int ns = std::min(K, 4 * (((m + BS_WAVES - 1) / BS_WAVES + 3) / 4));
                int vxmin = 1 << 20, vxmax = -(1 << 20), vymin = 1 << 20, vymax = -(1 << 20);
                for (int u = u0; u < u0 + m; ++u) {
                    vxmin = std::min(vxmin, U[u].first); vxmax = std::max(vxmax, U[u].first);
                    vymin = std::min(vymin, U[u].second); vymax = std::max(vymax, U[u].second);
                }
                // x0 even: region pairs (x, x + 1) never straddle column 0
                const int rx0 = (gx0 - vxmax) & ~1, ry0 = gy0 - vymax;
                const int rw = gx1 - vxmin - rx0 + 1, rh = gy1 - vymin - ry0 + 1;
                gitems.push_back({u0, m, ns, rx0, ry0, rw, rh});
                maxw = std::max(maxw, rw);
                maxh = std::max(maxh, rh);
            }
            if ((maxw + (maxw & 1)) * maxh <= bs_max_region(K)) break;
        }
        // One row pitch for all items of the group, even (the kernel moves
        // the region in pairs of columns).  A lane reads LDS at
        // (wy - ry0) pitch + (wx - rx0) - (slot offset), so the bank of
        // every gather follows key = (wx + pitch wy) mod 32 up to a shift
        // common to the wave.  A 64-bit LDS read serves 16 lanes per pass (32
        // on a 64-bank LDS): the pitch (one of the even values from the
        // widest region up to 8 more, within the LDS capacity) is the one
        // whose keys spread most evenly over the group
        // (at most 4 w per key mod 16, then 2 per key), and lanes are then
        // assigned so that each run of 16 lanes has distinct key mod 16 and,
        // where the keys allow, each run of 32 distinct key.
        int maxh = 0;
        for (const Item &gt : gitems) maxh = std::max(maxh, gt.rh);
        int pitch = maxw + (maxw & 1), best = 1 << 30;
        for (int cand = maxw + (maxw & 1); cand < maxw + 9; cand += 2) {
            if (cand * maxh > bs_max_region(K)) break;
            int c16[16] = {}, c32[32] = {};
            for (int i : gset) {
                const int key = ((pl->W[2 * i] + cand * pl->W[2 * i + 1]) % 32 + 32) % 32;
                ++c32[key];
                ++c16[key & 15];
            }
            int score = 0;
            for (int k = 0; k < 16; ++k) score += 4 * std::max(0, c16[k] - 4);
            for (int k = 0; k < 32; ++k) score += std::max(0, c32[k] - 2);
            if (score < best) { best = score; pitch = cand; }
        }
        int lane_w[BS_LANES];
        std::fill(lane_w, lane_w + BS_LANES, -1);
        {
            // bucket by key mod 16, each bucket alternating its two key
            // classes, dealt to the 4 runs of 16 lanes in order
            std::vector<std::vector<int>> bucket(16);
            for (int k16 = 0; k16 < 16; ++k16) {
                std::vector<int> a, b;
                for (int i : gset) {
                    const int key = ((pl->W[2 * i] + pitch * pl->W[2 * i + 1]) % 32 + 32) % 32;
                    if ((key & 15) == k16) (key < 16 ? a : b).push_back(i);
                }
                if (a.size() < b.size()) std::swap(a, b);
                for (size_t j = 0; j < a.size(); ++j) {
                    bucket[k16].push_back(a[j]);
                    if (j < b.size()) bucket[k16].push_back(b[j]);
                }
            }
            std::vector<int> rest;
            for (int k16 = 0; k16 < 16; ++k16) {
                for (size_t j = 0; j < bucket[k16].size(); ++j) {
                    if (j < 4) lane_w[16 * j + k16] = bucket[k16][j];
                    else rest.push_back(bucket[k16][j]);
                }
            }
            for (int lane = 0; lane < BS_LANES && !rest.empty(); ++lane)
                if (lane_w[lane] < 0) { lane_w[lane] = rest.back(); rest.pop_back(); }
        }
        std::vector<std::unordered_map<int, int>> rank(BS_LANES);
        for (int lane = 0; lane < BS_LANES; ++lane) {
            int i = lane_w[lane];
            if (i < 0) {
                // idle lane: repeat a w of its own 16-lane run (same address,
                // no extra bank conflict); its results are dropped
                for (int l = lane & ~15; l < (lane & ~15) + 16 && i < 0; ++l) i = lane_w[l];
                for (int l = 0; l < BS_LANES && i < 0; ++l) i = lane_w[l];
            } else {
                for (size_t j = 0; j < Sw[i].size() / 2; ++j)
                    rank[lane][(Sw[i][2 * j + 1] + 64) * 256 + (Sw[i][2 * j] + 64)] = (int)j;
            }
            pl->group_xy[((size_t)gi * BS_LANES + lane) * 2 + 0] = pl->W[2 * i];
            pl->group_xy[((size_t)gi * BS_LANES + lane) * 2 + 1] = pl->W[2 * i + 1];
        }
        for (const Item &gt : gitems) {
            const int u0 = gt.u0, m = gt.m, rx0 = gt.rx0, ry0 = gt.ry0, rw = pitch, rh = gt.rh;
            // the item's v in runs of 4 slots, dealt to the waves in turn (at
            // least one run each): wave c runs nsw[c] slots, the first of its
            // runs real, so an item of m v runs 4 ceil(m / 4) slots in all
            int nsw[BS_WAVES], cstart[BS_WAVES + 1];
            const int runs = std::max(BS_WAVES, (m + 3) / 4);
            cstart[0] = u0;
            for (int c = 0; c < BS_WAVES; ++c) {
                nsw[c] = 4 * (runs / BS_WAVES + (c < runs % BS_WAVES ? 1 : 0));
                cstart[c + 1] = cstart[c] + std::min(nsw[c], std::max(0, u0 + m - cstart[c]));
            }
            if (pitch * rh > bs_max_region(K)) { *err = "bispectrum region too large"; return false; }
            pl->max_region = std::max(pl->max_region, pitch * rh);
            int32_t it[BS_ITEM_INTS] = {gi, rx0, ry0, rw, rh, rw * rh, pitch, 0, nsw[0], nsw[1], nsw[2], nsw[3]};
            for (int wv = 0; wv < BS_WAVES; ++wv) {
                const int nreal = cstart[wv + 1] - cstart[wv];
                pl->computed_terms += (int64_t)nsw[wv] * BS_LANES;
                for (int k = 0; k < K; ++k) {
                    // slots past the real v of the chunk repeat the item's first v
                    const bool real = k < nreal;
                    const int u = real ? cstart[wv] + k : u0;
                    const int vx = U[u].first, vy = U[u].second;
                    pl->slot_v.push_back(vy * pitch + vx);
                    const uint32_t so = (uint32_t)((vy + 16) * N + (vx & (N - 1)));
                    pl->slot_v.push_back((int32_t)so);
                    for (int lane = 0; lane < BS_LANES; ++lane) {
                        int32_t o = -1;
                        if (real && lane_w[lane] >= 0) {
                            auto f = rank[lane].find((vy + 64) * 256 + (vx + 64));
                            if (f != rank[lane].end()) o = pl->woff[lane_w[lane]] + f->second;
                        }
                        if (o >= 0) ++covered;
                        pl->out_idx.push_back(o);
                    }
                }
            }
            pl->items.insert(pl->items.end(), it, it + BS_ITEM_INTS);
        }
    }
    pl->n_items = (int)(pl->items.size() / BS_ITEM_INTS);
    if (covered != pl->s_count) { *err = "internal: bispectrum work does not cover S"; return false; }

    // constant tables, computed in FP64 and rounded once
    const double pi = 3.14159265358979323846;
    pl->twiddle.resize(2 * N);
    for (int k = 0; k < N; ++k) {
        pl->twiddle[2 * k] = (float)std::cos(2.0 * pi * k / N);
        pl->twiddle[2 * k + 1] = (float)-std::sin(2.0 * pi * k / N);
    }
    pl->hann.resize(N);
    double hs = 0;
    for (int n = 0; n < N; ++n) {
        double h = 0.5 - 0.5 * std::cos(2.0 * pi * n / N);
        pl->hann[n] = (float)h;
        hs += h;
    }
    pl->hann_sum2 = hs * hs;
    pl->filt.resize(nW);
    for (int i = 0; i < nW; ++i) {
        double rho = std::hypot((double)pl->W[2 * i], (double)pl->W[2 * i + 1]) / (N / 2.0);
        rho = std::min(rho, 1.0);
        pl->filt[i] = (float)((2.0 / pi) * (std::acos(rho) - rho * std::sqrt(1.0 - rho * rho)));
    }
    return true;
}

}  // namespace nvsm
