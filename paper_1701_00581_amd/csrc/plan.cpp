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

    // sample indices are kept in 30 bits by the kernels' tables
    if (pl->s_count >= (int64_t)1 << 30) { *err = "bispectrum set too large"; return false; }

    // phasor window: inner entries |w| <= R, the rest in a ring; each
    // shell's lowest ring entry read comes from its sample codes
    pl->n_inner = 0;
    while (pl->n_inner < nW) {
        const int x = pl->W[2 * pl->n_inner], y = pl->W[2 * pl->n_inner + 1];
        if (x * x + y * y > R * R) break;
        ++pl->n_inner;
    }
    const int nshell = (int)pl->shell_wb.size() - 1;
    std::vector<int32_t> lo(nshell);
    int span = 1;
    for (int sh = 0; sh < nshell; ++sh) {
        int l = pl->shell_wb[sh];
        for (int32_t t = pl->woff[pl->shell_wb[sh]]; t < pl->woff[pl->shell_wb[sh + 1]]; ++t) {
            const int ia = (int)((pl->phase_code[t] >> 16) & 0x7fffu), ib = (int)(pl->phase_code[t] & 0x7fffu);
            if (ia >= pl->n_inner) l = std::min(l, ia);
            if (ib >= pl->n_inner) l = std::min(l, ib);
        }
        lo[sh] = std::max(l, pl->n_inner);
        span = std::max(span, pl->shell_wb[sh + 1] - lo[sh]);
    }
    pl->ring_size = span;
    pl->shell_ring_off.resize(nshell);
    for (int sh = 0; sh < nshell; ++sh)
        pl->shell_ring_off[sh] = (lo[sh] - pl->n_inner) / span * span;
    auto slot_of = [&](int i, int ro) {
        if (i < pl->n_inner) return i;
        int q = i - pl->n_inner - ro;
        if (q >= span) q -= span;
        return pl->n_inner + q;
    };
    pl->phase_slot_code.resize(pl->phase_code.size());
    pl->w_slot.resize(nW);
    for (int sh = 0; sh < nshell; ++sh) {
        const int ro = pl->shell_ring_off[sh];
        for (int w = pl->shell_wb[sh]; w < pl->shell_wb[sh + 1]; ++w) {
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

    // phase-solve units: shells 1.. cut into runs of SOLVE_WAVES w
    pl->solve_units.clear();
    pl->n_units = 0;
    for (int sh = 1; sh < nshell; ++sh) {
        for (int w0 = pl->shell_wb[sh]; w0 < pl->shell_wb[sh + 1]; w0 += SOLVE_WAVES) {
            const int last = w0 + SOLVE_WAVES >= pl->shell_wb[sh + 1];
            for (int j = 0; j < SOLVE_WAVES; ++j) {
                const int w = w0 + j;
                if (w < pl->shell_wb[sh + 1])
                    pl->solve_units.insert(pl->solve_units.end(),
                                           {w, pl->woff[w], (pl->woff[w + 1] - pl->woff[w]) | (last << 16), pl->w_slot[w]});
                else
                    pl->solve_units.insert(pl->solve_units.end(), {-1, 0, last << 16, 0});
            }
            ++pl->n_units;
        }
    }

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
    // union of their sets (the v slots a row of lanes runs) is little larger
    // than each set.  Groups: radial bands (8 wide up to 24, then about 10
    // wide), each sorted by angle and cut into equal groups of <= 64; each
    // row of 16 lanes (the rows of the DPP broadcast) takes about a quarter
    // of its group by angle and runs the union of its own 16 sets.  Wider
    // bands give narrower angles (fewer idle lanes) but larger staged
    // regions.
    std::vector<int> edges = {0};
    for (int e = 8; e <= 24; e += 8)
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
        // Rows: each run of 16 lanes (a row of the DPP broadcast) holds a
        // quarter of the group by angle and runs its own v: the union of S(w)
        // over 16 w of close direction is nearer each S(w) than the union over
        // all 64.
        const int ng = (int)gset.size();
        std::vector<int> rw[BS_ROWS];
        std::vector<std::pair<int, int>> U[BS_ROWS];   // (vx, vy) per row, sorted by (vy, vx)
        int bx0[BS_ROWS], bx1[BS_ROWS], by0[BS_ROWS], by1[BS_ROWS];
        size_t nUmax = 0;
        struct Item { int u0, m, rx0, ry0, rh; };
        std::vector<Item> gitems;
        int maxw = 0, maxh = 0;
        auto dummy = [&](int r, int u0) -> std::pair<int, int> {
            if (U[r].empty()) return {0, 0};
            return u0 < (int)U[r].size() ? U[r][u0] : U[r].back();
        };
        // The rows' unions, and items: item i takes positions [i mcap,
        // (i + 1) mcap) of every row's list.  A slot past a row's list runs
        // the row's dummy v (its chunk's first v, or its list's last once the
        // list is used up), which the staged region covers too.  Items hold
        // fewer v (in steps of 4 per wave) where the region of a full item
        // would not fit the LDS capacity.
        auto make_items = [&]() {
            nUmax = 0;
            for (int r = 0; r < BS_ROWS; ++r) {
                std::map<std::pair<int, int>, int> uni;  // (vy, vx)
                bx0[r] = by0[r] = 1 << 20;
                bx1[r] = by1[r] = -(1 << 20);
                U[r].clear();
                for (int i : rw[r]) {
                    const int wx = pl->W[2 * i], wy = pl->W[2 * i + 1];
                    bx0[r] = std::min(bx0[r], wx); bx1[r] = std::max(bx1[r], wx);
                    by0[r] = std::min(by0[r], wy); by1[r] = std::max(by1[r], wy);
                    for (size_t j = 0; j < Sw[i].size() / 2; ++j) uni[{Sw[i][2 * j + 1], Sw[i][2 * j]}] = 1;
                }
                for (auto &u : uni) U[r].push_back({u.first.second, u.first.first});
                nUmax = std::max(nUmax, U[r].size());
            }
            for (int mcap = BS_WAVES * K; mcap > 0; mcap -= 4 * BS_WAVES) {
                gitems.clear();
                maxw = maxh = 0;
                for (int u0 = 0; u0 < (int)nUmax; u0 += mcap) {
                    int m = 0, x0 = 1 << 20, x1 = -(1 << 20), y0 = 1 << 20, y1 = -(1 << 20);
                    for (int r = 0; r < BS_ROWS; ++r) {
                        if (rw[r].empty()) continue;
                        const int n = std::max(0, std::min((int)U[r].size() - u0, mcap));
                        m = std::max(m, n);
                        auto extend = [&](const std::pair<int, int> &v) {
                            x0 = std::min(x0, bx0[r] - v.first); x1 = std::max(x1, bx1[r] - v.first);
                            y0 = std::min(y0, by0[r] - v.second); y1 = std::max(y1, by1[r] - v.second);
                        };
                        for (int u = u0; u < u0 + n; ++u) extend(U[r][u]);
                        extend(dummy(r, u0));
                    }
                    // x0 even: region pairs (x, x + 1) never straddle column 0
                    x0 &= ~1;
                    gitems.push_back({u0, m, x0, y0, y1 - y0 + 1});
                    maxw = std::max(maxw, x1 - x0 + 1);
                    maxh = std::max(maxh, y1 - y0 + 1);
                }
                if ((maxw + (maxw & 1)) * maxh <= bs_max_region(K)) break;
            }
        };
        // One row pitch for all items of the group, even (the kernel moves
        // the region in pairs of columns).  A lane reads LDS at
        // (wy - ry0) pitch + (wx - rx0) - (its row's slot offset), so within
        // a row the bank of every gather follows key = (wx + pitch wy) mod 32
        // up to a shift common to the row.  A 64-bit LDS read serves one row
        // of 16 lanes per pass, so a row's lanes should hold distinct keys
        // mod 16.
        auto key_of = [&](int i, int pch) { return ((pl->W[2 * i] + pch * pl->W[2 * i + 1]) % 32 + 32) % 32; };
        auto collisions = [&](int pch) {
            int score = 0;
            for (int r = 0; r < BS_ROWS; ++r) {
                int c16[16] = {};
                for (int i : rw[r]) ++c16[key_of(i, pch) & 15];
                for (int k = 0; k < 16; ++k) score += std::max(0, c16[k] - 1);
            }
            return score;
        };
        // Rows by angle: quarters of the group (which is sorted by angle).
        auto angular_rows = [&]() {
            for (int r = 0; r < BS_ROWS; ++r) rw[r].clear();
            for (int j = 0; j < ng; ++j) rw[j * BS_ROWS / ng].push_back(gset[j]);
        };
        // Rows by angle with distinct keys: the w are taken in angle order
        // and each goes to the first row (from the current one on) whose
        // lanes do not hold its key mod 16 yet, else to the current row.
        auto keyed_rows = [&](int pch) {
            for (int r = 0; r < BS_ROWS; ++r) rw[r].clear();
            const int cap = (ng + BS_ROWS - 1) / BS_ROWS;
            int cur = 0;
            for (int j = 0; j < ng; ++j) {
                while (cur < BS_ROWS - 1 && (int)rw[cur].size() >= cap) ++cur;
                const int key = key_of(gset[j], pch) & 15;
                int dst = -1;
                for (int r = cur; r < BS_ROWS && dst < 0; ++r) {
                    if ((int)rw[r].size() >= cap) continue;
                    bool used = false;
                    for (int i : rw[r]) used |= (key_of(i, pch) & 15) == key;
                    if (!used) dst = r;
                }
                rw[dst < 0 ? cur : dst].push_back(gset[j]);
            }
        };
        angular_rows();
        make_items();
        // the pitch (an even value from the widest region up to 8 more,
        // within the LDS capacity) with the fewest repeated keys, for the
        // angular rows and for the keyed rows of that pitch; the keyed rows
        // are taken where their own regions fit that pitch
        int pitch = maxw + (maxw & 1), best = 1 << 30, best_keyed = -1;
        const int w_ang = maxw, h_ang = maxh;
        for (int cand = w_ang + (w_ang & 1); cand < w_ang + 9; cand += 2) {
            if (cand * h_ang > bs_max_region(K)) break;
            angular_rows();
            int sc = collisions(cand);
            if (sc < best) { best = sc; pitch = cand; best_keyed = 0; }
            keyed_rows(cand);
            sc = collisions(cand);
            if (sc < best) { best = sc; pitch = cand; best_keyed = 1; }
        }
        if (best_keyed == 1) {
            keyed_rows(pitch);
            make_items();
            if (maxw > pitch || pitch * maxh > bs_max_region(K)) {
                angular_rows();
                make_items();
                best_keyed = 0;
            }
        } else {
            angular_rows();
            make_items();
        }
        if (nUmax == 0) continue;
        int lane_w[BS_LANES];
        std::fill(lane_w, lane_w + BS_LANES, -1);
        for (int r = 0; r < BS_ROWS; ++r) {
            std::vector<int> rest;
            for (int i : rw[r]) {
                const int l = 16 * r + (key_of(i, pitch) & 15);
                if (lane_w[l] < 0) lane_w[l] = i;
                else rest.push_back(i);
            }
            for (int l = 16 * r; l < 16 * r + 16 && !rest.empty(); ++l)
                if (lane_w[l] < 0) { lane_w[l] = rest.back(); rest.pop_back(); }
        }
        std::vector<std::unordered_map<int, int>> rank(BS_LANES);
        for (int lane = 0; lane < BS_LANES; ++lane) {
            int i = lane_w[lane];
            if (i < 0) {
                // idle lane: repeat a w of its own row (same address, no extra
                // bank conflict); its results are dropped.  A row with no w
                // repeats the group's first.
                for (int l = lane & ~15; l < (lane & ~15) + 16 && i < 0; ++l) i = lane_w[l];
                if (i < 0) i = gset[0];
            } else {
                for (size_t j = 0; j < Sw[i].size() / 2; ++j)
                    rank[lane][(Sw[i][2 * j + 1] + 64) * 256 + (Sw[i][2 * j] + 64)] = (int)j;
            }
            pl->group_xy[((size_t)gi * BS_LANES + lane) * 2 + 0] = pl->W[2 * i];
            pl->group_xy[((size_t)gi * BS_LANES + lane) * 2 + 1] = pl->W[2 * i + 1];
        }
        for (const Item &gt : gitems) {
            const int u0 = gt.u0, m = gt.m, rx0 = gt.rx0, ry0 = gt.ry0, rh = gt.rh;
            // the item's v positions in runs of 4 slots, dealt to the waves in
            // turn (at least one run each): wave c runs nsw[c] slots, at
            // positions cstart[c] .. of every row's chunk
            int nsw[BS_WAVES], cstart[BS_WAVES + 1];
            const int runs = std::max(BS_WAVES, (m + 3) / 4);
            cstart[0] = u0;
            for (int c = 0; c < BS_WAVES; ++c) {
                nsw[c] = 4 * (runs / BS_WAVES + (c < runs % BS_WAVES ? 1 : 0));
                cstart[c + 1] = cstart[c] + nsw[c];
            }
            if (pitch * rh > bs_max_region(K)) { *err = "bispectrum region too large"; return false; }
            pl->max_region = std::max(pl->max_region, pitch * rh);
            int32_t it[BS_ITEM_INTS] = {gi, rx0, ry0, pitch, rh, pitch * rh, pitch, 0, nsw[0], nsw[1], nsw[2], nsw[3]};
            for (int wv = 0; wv < BS_WAVES; ++wv) {
                pl->computed_terms += (int64_t)nsw[wv] * BS_LANES;
                // the v of each row and slot (dummy past the row's chunk)
                std::pair<int, int> vs[BS_ROWS][BS_MAX_SLOTS];
                bool real[BS_ROWS][BS_MAX_SLOTS];
                for (int r = 0; r < BS_ROWS; ++r)
                    for (int k = 0; k < K; ++k) {
                        const int u = cstart[wv] + k;
                        real[r][k] = k < nsw[wv] && u < u0 + m && u < (int)U[r].size();
                        vs[r][k] = real[r][k] ? U[r][u] : dummy(r, u0);
                        const int vx = vs[r][k].first, vy = vs[r][k].second;
                        pl->slot_v.push_back(vy * pitch + vx);
                        pl->slot_v.push_back((int32_t)((vy + 16) * N + (vx & (N - 1))));
                    }
                for (int k = 0; k < K; ++k)
                    for (int lane = 0; lane < BS_LANES; ++lane) {
                        const int r = lane / 16;
                        int32_t o = -1;
                        if (real[r][k] && lane_w[lane] >= 0) {
                            auto f = rank[lane].find((vs[r][k].second + 64) * 256 + (vs[r][k].first + 64));
                            if (f != rank[lane].end()) o = pl->woff[lane_w[lane]] + f->second;
                        }
                        if (o >= 0) ++covered;
                        pl->out_idx.push_back(o);
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
