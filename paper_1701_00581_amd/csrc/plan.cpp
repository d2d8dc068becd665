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

    // Bispectrum work: 8x8 blocks of w; the union of their v, cut into
    // balanced chunks of <= K, BS_WAVES chunks per workgroup.
    const int half = N / 2;
    const int nbx = N / BS_BLOCK;
    std::map<std::pair<int, int>, std::vector<int>> blocks;  // (cy, cx) -> w ids
    for (int i = 0; i < nW; ++i) {
        int cx = (pl->W[2 * i] + half) / BS_BLOCK, cy = pl->W[2 * i + 1] / BS_BLOCK;
        blocks[{cy, cx}].push_back(i);
    }
    (void)nbx;
    pl->items.clear();
    pl->slot_v.clear();
    pl->out_idx.clear();
    pl->computed_terms = 0;
    int64_t covered = 0;
    for (auto &kv : blocks) {
        const int by0 = kv.first.first * BS_BLOCK;
        const int bx0 = kv.first.second * BS_BLOCK - half;
        // lane -> w id, and the rank of each v inside S(w)
        int lane_w[BS_LANES];
        std::fill(lane_w, lane_w + BS_LANES, -1);
        std::vector<std::unordered_map<int, int>> rank(BS_LANES);
        std::map<std::pair<int, int>, int> uni;  // (vy, vx) sorted union
        for (int i : kv.second) {
            int lane = (pl->W[2 * i + 1] - by0) * BS_BLOCK + (pl->W[2 * i] - bx0);
            lane_w[lane] = i;
            for (size_t j = 0; j < Sw[i].size() / 2; ++j) {
                int vx = Sw[i][2 * j], vy = Sw[i][2 * j + 1];
                rank[lane][(vy + 64) * 256 + (vx + 64)] = (int)j;
                uni[{vy, vx}] = 1;
            }
        }
        std::vector<std::pair<int, int>> U;  // (vx, vy)
        for (auto &u : uni) U.push_back({u.first.second, u.first.first});
        if (U.empty()) continue;
        const int nU = (int)U.size();
        const int nchunk = (nU + K - 1) / K;
        const int ngroup = (nchunk + BS_WAVES - 1) / BS_WAVES;
        // balanced chunk sizes
        std::vector<int> cstart(nchunk + 1, 0);
        for (int c = 0; c < nchunk; ++c) cstart[c + 1] = cstart[c] + nU / nchunk + (c < nU % nchunk ? 1 : 0);
        for (int g = 0; g < ngroup; ++g) {
            int c0 = g * BS_WAVES, c1 = std::min(nchunk, c0 + BS_WAVES);
            int vxmin = 1 << 20, vxmax = -(1 << 20), vymin = 1 << 20, vymax = -(1 << 20);
            for (int u = cstart[c0]; u < cstart[c1]; ++u) {
                vxmin = std::min(vxmin, U[u].first); vxmax = std::max(vxmax, U[u].first);
                vymin = std::min(vymin, U[u].second); vymax = std::max(vymax, U[u].second);
            }
            int rx0 = bx0 - vxmax, ry0 = by0 - vymax;
            int rw = (bx0 + BS_BLOCK - 1 - vxmin) - rx0 + 1;
            int rh = (by0 + BS_BLOCK - 1 - vymin) - ry0 + 1;
            const int pitch = bs_region_pitch(rw);
            if (pitch * rh > bs_region_cap(K)) { *err = "bispectrum region too large"; return false; }
            int32_t it[BS_ITEM_INTS] = {bx0, by0, rx0, ry0, rw, rh, rw * rh, pitch, 0, 0, 0, 0};
            for (int wv = 0; wv < BS_WAVES; ++wv) {
                int c = c0 + wv;
                int ns = c < c1 ? cstart[c + 1] - cstart[c] : 0;
                it[8 + wv] = ns;
                pl->computed_terms += (int64_t)ns * BS_LANES;
                for (int k = 0; k < K; ++k) {
                    int u = k < ns ? cstart[c] + k : cstart[c0];
                    int vx = U[u].first, vy = U[u].second;
                    pl->slot_v.push_back(vy * pitch + vx);
                    const uint32_t so = (uint32_t)((vy + 16) * N + (vx & (N - 1)));
                    pl->slot_v.push_back((int32_t)so);
                    for (int lane = 0; lane < BS_LANES; ++lane) {
                        int32_t o = -1;
                        if (k < ns && lane_w[lane] >= 0) {
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
