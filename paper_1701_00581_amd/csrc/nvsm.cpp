// C-ABI of the speckle-masking library: context, validation, plan cache,
// workspace layout and the launch sequence on the caller's stream.
#include "nvsm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"
#include "scratch.hpp"

using namespace nvsm;

namespace {

constexpr int CHUNK_FRAMES = 20;     // frames per ingest workgroup (even)
constexpr size_t ALIGN = 256;
constexpr size_t QUEUE_BYTES = 256;  // 8 int counters, padded to the alignment

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct DevicePlan {
    HostPlan h;
    int max_sw = 0;
    std::vector<void *> bufs;
    int *W = nullptr, *woff = nullptr, *w_slot = nullptr, *items = nullptr, *units = nullptr,
        *group_xy = nullptr, *slot = nullptr, *out_idx = nullptr, *lsq_fin = nullptr;
    unsigned *code = nullptr, *wcode = nullptr;
    float2 *twiddle = nullptr;
    float *hann = nullptr, *filt = nullptr;
    ~DevicePlan() {
        for (void *p : bufs) (void)hipFree(p);
    }
};

}  // namespace

constexpr int NSTAGE = 4;
enum { ST_INGEST = 0, ST_BISPEC = 1, ST_SOLVE = 2, ST_SYNTH = 3 };

struct nvsm_context {
    int device = 0;
    std::string err;
    // plans by (N, u_cut, v_radius, slots per wave)
    std::map<std::tuple<int, int, int, int>, std::unique_ptr<DevicePlan>> plans;
    // launch choices by (N, u_cut, v_radius): slots per wave, bispectrum form
    std::map<std::tuple<int, int, int>, std::pair<int, int>> tuned;
    // stage timing
    bool prof = false;
    std::vector<hipEvent_t> free_ev;
    struct Rec { int stage; hipEvent_t a, b; };
    std::vector<Rec> recs;
    ~nvsm_context() {
        for (auto &r : recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
        for (auto e : free_ev) (void)hipEventDestroy(e);
    }
};

namespace {

nvsm_status fail(nvsm_context *ctx, nvsm_status s, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return s;
}

nvsm_status check_params(const nvsm_params *p, std::string *msg) {
    if (!p) { *msg = "params is NULL"; return NVSM_ERR_INVALID_ARG; }
    if (p->patch != 64 && p->patch != 128) { *msg = "patch must be 64 or 128"; return NVSM_ERR_INVALID_ARG; }
    if (p->stride < 1 || p->stride > p->patch) { *msg = "stride must be in [1, patch]"; return NVSM_ERR_INVALID_ARG; }
    if (p->u_cut < 2 || p->u_cut >= p->patch / 2) { *msg = "u_cut must be in [2, patch/2)"; return NVSM_ERR_INVALID_ARG; }
    if (p->v_radius < 1 || p->v_radius > 16 || p->v_radius >= p->u_cut) {
        *msg = "v_radius must be in [1, min(16, u_cut))";
        return NVSM_ERR_INVALID_ARG;
    }
    if (p->window != 0 && p->window != 1) { *msg = "window must be 0 or 1"; return NVSM_ERR_INVALID_ARG; }
    if (p->phase_method != 0 && p->phase_method != 1) { *msg = "phase_method must be 0 or 1"; return NVSM_ERR_NOT_IMPLEMENTED; }
    if (p->phase_method == 1 && (p->lsq_iters < 1 || p->lsq_iters > 10000)) {
        *msg = "lsq_iters must be in [1, 10000]";
        return NVSM_ERR_INVALID_ARG;
    }
    if (p->noise_bias < 0 || p->noise_bias > 2) { *msg = "noise_bias must be 0, 1 or 2"; return NVSM_ERR_INVALID_ARG; }
    if (p->noise_bias == 2 && !(p->photons_per_adu > 0.0 && std::isfinite(p->photons_per_adu))) {
        *msg = "photons_per_adu must be finite and > 0";
        return NVSM_ERR_INVALID_ARG;
    }
    if (p->filter != 0 && p->filter != 1) { *msg = "filter must be 0 or 1"; return NVSM_ERR_INVALID_ARG; }
    if (!(p->stf_floor >= 0.0) || !std::isfinite(p->stf_floor)) { *msg = "stf_floor must be finite and >= 0"; return NVSM_ERR_INVALID_ARG; }
    return NVSM_OK;
}

nvsm_status check_shape(const nvsm_params *p, int H, int W, int F, std::string *msg) {
    if (F < 1) { *msg = "F must be >= 1"; return NVSM_ERR_SHAPE; }
    // the bispectrum kernel addresses one patch's F spectrum records
    // (rows -16 .. N/2-1 of N complex64) with 32-bit byte offsets
    if ((int64_t)F * (p->patch / 2 + 16) * p->patch * 8 > (int64_t)INT32_MAX) {
        *msg = "too many frames in one call: F * (N/2 + 16) * N * 8 must stay below 2^31";
        return NVSM_ERR_SHAPE;
    }
    if (H < p->patch || W < p->patch) { *msg = "frames smaller than a patch"; return NVSM_ERR_SHAPE; }
    if ((int64_t)H * W > ((int64_t)1 << 31) - 1) { *msg = "frame too large"; return NVSM_ERR_SHAPE; }
    return NVSM_OK;
}

struct Sizes {
    int64_t P = 0, nW = 0, S = 0, records = 0, wgs = 0;
    size_t spectra = 0, ppart = 0, mpart = 0, mupart = 0;      // accumulate scratch
    size_t cpart = 0, spart = 0, cw = 0, nbar = 0;             // photon-noise terms (noise_bias 2)
    size_t queue = 0;                                          // work-queue counters of this call
    size_t power = 0, mean = 0, mu = 0, bispec = 0, amp = 0, phasor = 0, patches = 0;
};

// One burst as the entry points receive it.
struct BurstIn {
    const void *frames = nullptr;
    int F = 0, H = 0, W = 0;
    int64_t pitch = 0;
    const double *stf = nullptr;
    float *out = nullptr;
};

// Numbers the patches, ingest workgroups, spectrum records and output
// pixels of up to MAX_BURSTS bursts consecutively.
void make_table(const nvsm_params *p, const BurstIn *in, int n, BurstTable *bt, int64_t *records) {
    *bt = BurstTable();
    bt->nb = n;
    int64_t P = 0, wgs = 0, rec = 0, pix = 0;
    for (int i = 0; i < n; ++i) {
        Tiling t;
        make_tiling(in[i].H, in[i].W, p->patch, p->stride, &t);
        BurstDesc &d = bt->b[i];
        d.frames = in[i].frames; d.pitch = in[i].pitch; d.stf = in[i].stf; d.out = in[i].out;
        d.F = in[i].F; d.H = in[i].H; d.W = in[i].W; d.ny = t.ny; d.nx = t.nx;
        d.patch0 = (int)P; d.ingest0 = (int)wgs; d.spec0 = rec; d.pix0 = pix;
        const int64_t Pb = (int64_t)t.ny * t.nx;
        P += Pb;
        wgs += Pb * ((in[i].F + CHUNK_FRAMES - 1) / CHUNK_FRAMES);
        rec += Pb * in[i].F;
        pix += (int64_t)in[i].H * in[i].W;
    }
    bt->patches = (int)P;
    bt->ingest_wgs = (int)wgs;
    bt->pixels = pix;
    *records = rec;
}

void sizes_for(int N, const BurstTable &bt, int64_t records, int64_t nW, int64_t S, Sizes *z, bool photon) {
    z->P = bt.patches;
    z->nW = nW;
    z->S = S;
    z->records = records;
    z->wgs = bt.ingest_wgs;
    z->spectra = align_up((size_t)records * (N / 2 + 16) * N * 8);   // rows -16 .. N/2-1
    z->ppart = align_up((size_t)z->wgs * (N / 2 + 1) * N * 4);
    z->mpart = align_up((size_t)z->wgs * 4 * 4);
    z->mupart = align_up((size_t)z->wgs * 4);
    z->power = align_up((size_t)z->P * N * N * 4);
    z->mean = align_up((size_t)z->P * 4 * 4);
    z->mu = align_up((size_t)z->P * 4);
    z->bispec = align_up((size_t)z->P * S * 8);
    z->amp = align_up((size_t)z->P * nW * 8);
    z->phasor = align_up((size_t)z->P * nW * 16);
    z->patches = align_up((size_t)z->P * N * N * 4);
    z->queue = QUEUE_BYTES;
    if (photon) {
        z->cpart = align_up((size_t)z->wgs * (N / 2 + 1) * N * 8);
        z->spart = align_up((size_t)z->wgs * 2 * 4);
        z->cw = align_up((size_t)z->P * (N / 2 + 16) * N * 8);
        z->nbar = align_up((size_t)z->P * 2 * 4);
    }
}

size_t ws_acc(const Sizes &z) {
    return z.spectra + z.ppart + z.mpart + z.mupart + z.cpart + z.spart + z.cw + z.nbar + z.queue;
}

// The persistent bispectrum's 8 work-queue counters live in the call's own
// workspace (after the rest of the accumulate scratch), so calls on
// different streams with different workspaces never share them.
int *queue_of(char *acc_ws, const Sizes &z) { return (int *)(acc_ws + ws_acc(z) - z.queue); }
size_t ws_rec(const Sizes &z) {
    return z.power + z.mean + z.mu + z.bispec + z.amp + z.phasor + z.patches + ws_acc(z);
}

// The streaming calls always run this many slots per wave, so the state's
// layout (the kernel's lane order) does not depend on the launch choice.
constexpr int STREAM_SLOTS = 16;

// Streaming buffers.  The state of one burst holds the running
// (sum, compensation) pairs: the bispectrum terms in the kernel's lane order
// (every computed slot of every item), then the power rows, mean spectrum
// and mean level.  The workspace of one stream holds the final means (the
// bispectrum in S order first), the solve and synthesis buffers, then the
// scratch for one group of frames.
struct StreamSizes {
    size_t acc_s = 0, acc_c = 0, psc = 0, msc = 0, musc = 0, csc = 0, ssc = 0;   // state
    size_t bis = 0, power = 0, mean = 0, mu = 0, amp = 0, phasor = 0, patches = 0, group = 0;   // workspace
    size_t state() const { return acc_s + acc_c + psc + msc + musc + csc + ssc; }
    size_t ws() const { return bis + power + mean + mu + amp + phasor + patches + group; }
};

// noise: the state also carries the photon-noise sums (noise_bias 2)
void stream_sizes(int N, int64_t P, int64_t nW, int64_t S, int64_t lane_terms, size_t group, StreamSizes *z,
                  bool noise = false) {
    const int64_t NP = (N / 2 + 1) * N;
    z->acc_s = align_up((size_t)P * lane_terms * 8);
    z->acc_c = align_up((size_t)P * lane_terms * 8);
    z->psc = align_up((size_t)P * NP * 8);
    z->msc = align_up((size_t)P * 4 * 8);
    z->musc = align_up((size_t)P * 8);
    z->csc = noise ? align_up((size_t)P * NP * 16) : 0;       // C: (sum, compensation) of re and im
    z->ssc = noise ? align_up((size_t)P * 4 * 4) : 0;         // q0 and T: (sum, compensation)
    z->bis = align_up((size_t)P * S * 8);
    z->power = align_up((size_t)P * N * N * 4);
    z->mean = align_up((size_t)P * 4 * 4);
    z->mu = align_up((size_t)P * 4);
    z->amp = align_up((size_t)P * nW * 8);
    z->phasor = align_up((size_t)P * nW * 16);
    z->patches = align_up((size_t)P * N * N * 4);
    z->group = group;
}

struct StreamView {
    float2 *acc_s, *acc_c, *psc, *msc, *musc;            // state
    float4 *csc;                                          // photon-noise sums (noise_bias 2)
    float *ssc;
    float2 *bis;                                          // workspace
    float *power, *mean, *mu;
    double *amp, *phasor;
    float *patches;
    char *group;
};

StreamView stream_view(char *st, char *ws, const StreamSizes &z) {
    StreamView v{};
    if (st) {
        v.acc_s = (float2 *)st; st += z.acc_s;
        v.acc_c = (float2 *)st; st += z.acc_c;
        v.psc = (float2 *)st; st += z.psc;
        v.msc = (float2 *)st; st += z.msc;
        v.musc = (float2 *)st; st += z.musc;
        v.csc = z.csc ? (float4 *)st : nullptr; st += z.csc;
        v.ssc = z.ssc ? (float *)st : nullptr;
    }
    v.bis = (float2 *)ws; ws += z.bis;
    v.power = (float *)ws; ws += z.power;
    v.mean = (float *)ws; ws += z.mean;
    v.mu = (float *)ws; ws += z.mu;
    v.amp = (double *)ws; ws += z.amp;
    v.phasor = (double *)ws; ws += z.phasor;
    v.patches = (float *)ws; ws += z.patches;
    v.group = ws;
    return v;
}

void count_sets(const nvsm_params *p, int64_t *nW, int64_t *S, int *shells) {
    std::vector<int32_t> w, wv;
    enumerate_W(p->u_cut, &w);
    enumerate_S(p->u_cut, p->v_radius, &wv);
    *nW = (int64_t)w.size() / 2;
    *S = (int64_t)wv.size() / 4;
    *shells = count_shells(w);
}

template <typename T>
nvsm_status upload(DevicePlan *dp, const std::vector<T> &v, T **out, std::string *msg) {
    void *d = nullptr;
    size_t bytes = std::max<size_t>(v.size() * sizeof(T), 4);
    if (hipMalloc(&d, bytes) != hipSuccess) { *msg = "hipMalloc failed for a table"; return NVSM_ERR_OOM; }
    dp->bufs.push_back(d);
    if (!v.empty() && hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
        *msg = "table upload failed";
        return NVSM_ERR_HIP;
    }
    *out = (T *)d;
    return NVSM_OK;
}

// Launch choices for p: the tuned ones if nvsm_autotune ran, else 16
// slots per wave and one workgroup per item.
std::pair<int, int> choice_of(const nvsm_context *ctx, const nvsm_params *p) {
    auto f = ctx->tuned.find(std::make_tuple(p->patch, p->u_cut, p->v_radius));
    return f == ctx->tuned.end() ? std::make_pair(16, 0) : f->second;
}

nvsm_status get_plan(nvsm_context *ctx, const nvsm_params *p, int slots, DevicePlan **out) {
    auto key = std::make_tuple(p->patch, p->u_cut, p->v_radius, slots);
    auto f = ctx->plans.find(key);
    if (f != ctx->plans.end()) { *out = f->second.get(); return NVSM_OK; }
    std::unique_ptr<DevicePlan> dp;
    try {
        dp.reset(new DevicePlan());
    } catch (const std::bad_alloc &) {
        return fail(ctx, NVSM_ERR_OOM, "host allocation failed");
    }
    std::string msg;
    try {
        if (!build_plan(p->patch, p->u_cut, p->v_radius, slots, &dp->h, &msg)) return fail(ctx, NVSM_ERR_INVALID_ARG, msg);
    } catch (const std::bad_alloc &) {
        return fail(ctx, NVSM_ERR_OOM, "host allocation failed while planning");
    }
    const HostPlan &h = dp->h;
    dp->max_sw = h.max_sw;
    if (h.solve_code.empty() || h.n_inner > 512 || h.ring_size > 3072)
        return fail(ctx, NVSM_ERR_INVALID_ARG, "sample count or phasor window too large for the phase kernel");
    if (h.n_inner + h.lsq_span > LSQ_ACC)
        return fail(ctx, NVSM_ERR_INVALID_ARG, "least-squares accumulator window too large");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, NVSM_ERR_HIP, "hipSetDevice failed");
    nvsm_status s;
    std::vector<float2> tw(h.N);
    for (int k = 0; k < h.N; ++k) tw[k] = make_float2(h.twiddle[2 * k], h.twiddle[2 * k + 1]);
    if ((s = upload(dp.get(), h.W, &dp->W, &msg)) ||
        (s = upload(dp.get(), h.woff, &dp->woff, &msg)) ||
        (s = upload(dp.get(), h.w_slot, &dp->w_slot, &msg)) ||
        (s = upload(dp.get(), h.solve_units, &dp->units, &msg)) ||
        (s = upload(dp.get(), h.solve_code, &dp->code, &msg)) ||
        (s = upload(dp.get(), h.phase_code, &dp->wcode, &msg)) ||
        (s = upload(dp.get(), h.lsq_fin, &dp->lsq_fin, &msg)) ||
        (s = upload(dp.get(), h.items, &dp->items, &msg)) ||
        (s = upload(dp.get(), h.group_xy, &dp->group_xy, &msg)) ||
        (s = upload(dp.get(), h.slot_v, &dp->slot, &msg)) ||
        (s = upload(dp.get(), h.out_idx, &dp->out_idx, &msg)) ||
        (s = upload(dp.get(), tw, &dp->twiddle, &msg)) ||
        (s = upload(dp.get(), h.hann, &dp->hann, &msg)) ||
        (s = upload(dp.get(), h.filt, &dp->filt, &msg)))
        return fail(ctx, s, msg);
    *out = dp.get();
    ctx->plans[key] = std::move(dp);
    return NVSM_OK;
}

nvsm_status get_plan(nvsm_context *ctx, const nvsm_params *p, DevicePlan **out) {
    return get_plan(ctx, p, choice_of(ctx, p).first, out);
}

// The plan of p's launch choice if it already exists (no allocation).
DevicePlan *find_plan(const nvsm_context *ctx, const nvsm_params *p) {
    auto f = ctx->plans.find(std::make_tuple(p->patch, p->u_cut, p->v_radius, choice_of(ctx, p).first));
    return f == ctx->plans.end() ? nullptr : f->second.get();
}

// Records an event pair around one stage when profiling is on.
struct StageTimer {
    nvsm_context *ctx;
    int stage;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    StageTimer(nvsm_context *c, int s, hipStream_t stream) : ctx(c), stage(s), st(stream) {
        if (!ctx || !ctx->prof) return;
        a = take();
        b = take();
        if (a && b) (void)hipEventRecord(a, st);
    }
    hipEvent_t take() {
        if (!ctx->free_ev.empty()) { hipEvent_t e = ctx->free_ev.back(); ctx->free_ev.pop_back(); return e; }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    ~StageTimer() {
        if (!ctx || !ctx->prof) return;
        if (a && b && hipEventRecord(b, st) == hipSuccess) { ctx->recs.push_back({stage, a, b}); return; }
        if (a) ctx->free_ev.push_back(a);
        if (b) ctx->free_ev.push_back(b);
    }
};

// 4-pixel vector loads need every quad of a patch row aligned to its size.
bool vec_ok(const nvsm_params *p, const BurstTable &bt, size_t px_bytes) {
    for (int i = 0; i < bt.nb; ++i) {
        const BurstDesc &d = bt.b[i];
        if (p->stride % 4 || (d.W - p->patch) % 4 || d.pitch % 4 || ((uintptr_t)d.frames % (4 * px_bytes)))
            return false;
    }
    return true;
}

// The bispectrum launch of a table over its accumulate scratch ws.
BispecArgs bispec_args(nvsm_context *ctx, DevicePlan *dp, const nvsm_params *p, const BurstTable &bt, const Sizes &z,
                       float *bispec, char *ws) {
    BispecArgs b;
    b.N = p->patch; b.bt = bt; b.spectra = (const float2 *)ws;
    b.n_items = dp->h.n_items; b.slots = dp->h.slots; b.items = dp->items; b.group_xy = dp->group_xy;
    b.slot_v = dp->slot; b.out_idx = dp->out_idx;
    b.bispec = (float2 *)bispec; b.s_count = z.S;
    b.form = choice_of(ctx, p).second; b.queue = queue_of(ws, z);
    if (p->noise_bias == 2) {
        // the photon-noise terms' place in the scratch (see run_accumulate)
        char *q = ws + z.spectra + z.ppart + z.mpart + z.mupart + z.cpart + z.spart;
        b.acc.noise_c = (const float2 *)q;
        b.acc.noise_t = (const float *)(q + z.cw);
    }
    return b;
}

hipError_t run_accumulate(nvsm_context *ctx, DevicePlan *dp, const nvsm_params *p, const BurstTable &bt,
                          const Sizes &z, nvsm_dtype dtype, float *power, float *mean_spec, float *mu,
                          float *bispec, char *ws, hipStream_t st) {
    IngestArgs a;
    a.N = p->patch;
    a.f32 = dtype == NVSM_F32;
    a.bt = bt;
    a.stride = p->stride;
    a.chunk_frames = CHUNK_FRAMES; a.window = p->window;
    a.vec = vec_ok(p, bt, a.f32 ? 4 : 2);
    a.inv_wsum = (float)(1.0 / (p->window ? dp->h.hann_sum2 : (double)p->patch * p->patch));
    a.twiddle = dp->twiddle; a.hann = dp->hann;
    a.spectra = (float2 *)ws;
    a.ppart = (float *)(ws + z.spectra);
    a.mpart = (float *)(ws + z.spectra + z.ppart);
    a.mupart = (float *)(ws + z.spectra + z.ppart + z.mpart);
    a.power = power; a.mean_spec = mean_spec; a.mu = mu;
    hipError_t e;
    NoiseArgs na;
    if (p->noise_bias == 2) {
        char *q = ws + z.spectra + z.ppart + z.mpart + z.mupart;
        na.in = a;
        na.inv_gain = (float)(1.0 / p->photons_per_adu);
        na.cpart = (float2 *)q; q += z.cpart;
        na.spart = (float *)q; q += z.spart;
        na.cgrid = (float2 *)q; q += z.cw;
        na.nbar = (float *)q;
    }
    {
        StageTimer t(ctx, ST_INGEST, st);
        e = launch_ingest(a, st);
        if (e == hipSuccess && p->noise_bias == 2) e = launch_noise(na, st);
    }
    if (e != hipSuccess || bispec == nullptr) return e;
    StageTimer t(ctx, ST_BISPEC, st);
    return launch_bispec(bispec_args(ctx, dp, p, bt, z, bispec, ws), st);
}

hipError_t run_solve(nvsm_context *ctx, DevicePlan *dp, const nvsm_params *p, const BurstTable &bt,
                     const float *power, const float *mean_spec, const float *bispec, double *amp,
                     double *phasor, hipStream_t st) {
    SolveArgs a;
    a.N = p->patch; a.bt = bt; a.nW = (int)(dp->h.W.size() / 2);
    a.max_sw = dp->max_sw; a.woff = dp->woff; a.Wxy = dp->W; a.code = dp->code;
    a.zero_slot = dp->h.zero_slot;
    a.w_slot = dp->w_slot; a.n_inner = dp->h.n_inner; a.ring = dp->h.ring_size;
    a.units = dp->units; a.n_units = dp->h.n_units;
    a.power = power; a.mean_spec = mean_spec; a.bispec = (const float2 *)bispec; a.s_count = dp->h.s_count;
    a.floor = p->stf_floor; a.noise_bias = p->noise_bias == 1; a.amp = amp;
    a.phasor = (double2 *)phasor;
    a.phase_method = p->phase_method; a.lsq_iters = p->lsq_iters;
    a.wcode = dp->wcode; a.lsq_fin = dp->lsq_fin;
    StageTimer t(ctx, ST_SOLVE, st);
    return launch_solve(a, st);
}

hipError_t run_synth(nvsm_context *ctx, DevicePlan *dp, const nvsm_params *p, const BurstTable &bt,
                     const double *amp, const double *phasor, const float *mu, float *patch_buf, bool mosaic,
                     hipStream_t st) {
    SynthArgs a;
    a.N = p->patch; a.bt = bt; a.nW = (int)(dp->h.W.size() / 2); a.window = p->window; a.Wxy = dp->W;
    a.amp = amp; a.phasor = (const double2 *)phasor; a.filt = p->filter ? dp->filt : nullptr;
    a.mu = mu; a.hann = dp->hann; a.twiddle = dp->twiddle; a.patch_buf = patch_buf;
    a.stride = p->stride; a.mosaic = mosaic;
    StageTimer t(ctx, ST_SYNTH, st);
    return launch_synth(a, st);
}

// The whole path for the bursts of one table, in a workspace laid out as
// power, mean spectrum, mean level, bispectrum, modulus, phasors,
// subimages, then the accumulate scratch.
hipError_t run_reconstruct(nvsm_context *ctx, DevicePlan *dp, const nvsm_params *p, const BurstTable &bt,
                           const Sizes &z, nvsm_dtype dtype, char *w, hipStream_t st) {
    float *power = (float *)w; w += z.power;
    float *mean = (float *)w; w += z.mean;
    float *mu = (float *)w; w += z.mu;
    float *bis = (float *)w; w += z.bispec;
    double *amp = (double *)w; w += z.amp;
    double *ph = (double *)w; w += z.phasor;
    float *pat = (float *)w; w += z.patches;
    hipError_t e = run_accumulate(ctx, dp, p, bt, z, dtype, power, mean, mu, bis, w, st);
    if (e != hipSuccess) return e;
    e = run_solve(ctx, dp, p, bt, power, mean, bis, amp, ph, st);
    if (e != hipSuccess) return e;
    return run_synth(ctx, dp, p, bt, amp, ph, mu, pat, true, st);
}

nvsm_status hip_fail(nvsm_context *ctx, hipError_t e, const char *where) {
    return fail(ctx, NVSM_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

// The transform kernels address a patch's pixels in a frame with 32-bit
// byte offsets from the patch origin: N rows of row_pitch elements of up
// to 4 bytes must stay below 2^32.
int64_t max_row_pitch(int N) { return ((int64_t)1 << 30) / N; }

nvsm_status check_burst(const nvsm_params *p, const BurstIn &bi, std::string *msg) {
    nvsm_status s = check_shape(p, bi.H, bi.W, bi.F, msg);
    if (s != NVSM_OK) return s;
    if (bi.pitch < bi.W) { *msg = "row_pitch < W"; return NVSM_ERR_SHAPE; }
    if (bi.pitch > max_row_pitch(p->patch)) { *msg = "row_pitch too large (N * row_pitch must stay below 2^30)"; return NVSM_ERR_SHAPE; }
    return NVSM_OK;
}

// Validates one burst and builds its table and sizes.
nvsm_status prepare_call(nvsm_context *ctx, const nvsm_params *p, const BurstIn &bi, DevicePlan **dp,
                         BurstTable *bt, Sizes *z) {
    std::string msg;
    nvsm_status s = check_params(p, &msg);
    if (s != NVSM_OK) return fail(ctx, s, msg);
    if ((s = check_burst(p, bi, &msg)) != NVSM_OK) return fail(ctx, s, msg);
    if ((s = get_plan(ctx, p, dp)) != NVSM_OK) return s;
    int64_t rec;
    make_table(p, &bi, 1, bt, &rec);
    sizes_for(p->patch, *bt, rec, (int64_t)((*dp)->h.W.size() / 2), (*dp)->h.s_count, z, p->noise_bias == 2);
    return NVSM_OK;
}

}  // namespace

extern "C" {

nvsm_status nvsm_create(int hip_device, nvsm_context **out) {
    if (!out) return NVSM_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return NVSM_ERR_HIP;
    if (hip_device < 0 || hip_device >= n) return NVSM_ERR_INVALID_ARG;
    // the no-allocation entry point's scratch array on this device
    if (scratch_setup(hip_device) != hipSuccess) return NVSM_ERR_HIP;
    nvsm_context *c = new (std::nothrow) nvsm_context();
    if (!c) return NVSM_ERR_OOM;
    c->device = hip_device;
    *out = c;
    return NVSM_OK;
}

void nvsm_destroy(nvsm_context *ctx) { delete ctx; }

const char *nvsm_status_string(nvsm_status s) {
    switch (s) {
        case NVSM_OK: return "ok";
        case NVSM_ERR_INVALID_ARG: return "invalid argument";
        case NVSM_ERR_SHAPE: return "shape mismatch";
        case NVSM_ERR_WORKSPACE: return "workspace too small";
        case NVSM_ERR_OOM: return "out of memory";
        case NVSM_ERR_HIP: return "HIP error";
        case NVSM_ERR_NOT_IMPLEMENTED: return "not implemented";
    }
    return "unknown status";
}

const char *nvsm_last_error(const nvsm_context *ctx) { return ctx ? ctx->err.c_str() : ""; }

nvsm_status nvsm_default_params(int32_t patch, nvsm_params *out) {
    if (!out || (patch != 64 && patch != 128)) return NVSM_ERR_INVALID_ARG;
    out->patch = patch;
    out->stride = patch / 2;
    out->u_cut = patch / 2 - 1;
    out->v_radius = 10;
    out->window = 1;
    out->phase_method = 0;
    out->noise_bias = 0;
    out->filter = 0;
    out->stf_floor = 1e-6;
    out->lsq_iters = 10;
    out->reserved = 0;
    out->photons_per_adu = 1.0;
    return NVSM_OK;
}

nvsm_status nvsm_plan(const nvsm_params *p, int32_t H, int32_t W, int32_t F, nvsm_plan_info *out) {
    std::string msg;
    if (!out) return NVSM_ERR_INVALID_ARG;
    nvsm_status s = check_params(p, &msg);
    if (s != NVSM_OK) return s;
    if ((s = check_shape(p, H, W, F, &msg)) != NVSM_OK) return s;
    int64_t nW, S;
    int shells;
    try {
        count_sets(p, &nW, &S, &shells);
    } catch (const std::bad_alloc &) {
        return NVSM_ERR_OOM;
    }
    BurstIn bi;
    bi.F = F; bi.H = H; bi.W = W; bi.pitch = W;
    BurstTable bt;
    int64_t rec;
    make_table(p, &bi, 1, &bt, &rec);
    Sizes z;
    sizes_for(p->patch, bt, rec, nW, S, &z, p->noise_bias == 2);
    out->patches_y = bt.b[0].ny;
    out->patches_x = bt.b[0].nx;
    out->patches = z.P;
    out->w_count = nW;
    out->s_count = S;
    out->shells = shells;
    out->frame_chunks = (F + CHUNK_FRAMES - 1) / CHUNK_FRAMES;
    out->ws_accumulate = ws_acc(z);
    out->ws_solve = 0;
    out->ws_synthesize = z.patches;
    out->ws_reconstruct = ws_rec(z);
    return NVSM_OK;
}

nvsm_status nvsm_w_index(const nvsm_params *p, int32_t *w, int64_t w_count) {
    std::string msg;
    if (!w) return NVSM_ERR_INVALID_ARG;
    nvsm_status s = check_params(p, &msg);
    if (s != NVSM_OK) return s;
    std::vector<int32_t> v;
    enumerate_W(p->u_cut, &v);
    if ((int64_t)v.size() / 2 != w_count) return NVSM_ERR_SHAPE;
    std::memcpy(w, v.data(), v.size() * sizeof(int32_t));
    return NVSM_OK;
}

nvsm_status nvsm_bispectrum_index(const nvsm_params *p, int32_t *wv, int64_t s_count) {
    std::string msg;
    if (!wv) return NVSM_ERR_INVALID_ARG;
    nvsm_status s = check_params(p, &msg);
    if (s != NVSM_OK) return s;
    std::vector<int32_t> v;
    enumerate_S(p->u_cut, p->v_radius, &v);
    if ((int64_t)v.size() / 4 != s_count) return NVSM_ERR_SHAPE;
    std::memcpy(wv, v.data(), v.size() * sizeof(int32_t));
    return NVSM_OK;
}

nvsm_status nvsm_prepare(nvsm_context *ctx, const nvsm_params *p) {
    if (!ctx) return NVSM_ERR_INVALID_ARG;
    std::string msg;
    nvsm_status s = check_params(p, &msg);
    if (s != NVSM_OK) return fail(ctx, s, msg);
    DevicePlan *dp;
    return get_plan(ctx, p, &dp);
}

nvsm_status nvsm_accumulate(nvsm_context *ctx, const nvsm_params *p, const void *frames, nvsm_dtype dtype,
                            int32_t F, int32_t H, int32_t W, int64_t row_pitch, float *power,
                            float *mean_spec, float *mu, float *bispec, void *workspace,
                            size_t workspace_bytes, void *stream) {
    if (!ctx) return NVSM_ERR_INVALID_ARG;
    if (!frames || !power || !mean_spec || !mu) return fail(ctx, NVSM_ERR_INVALID_ARG, "null buffer");
    if (dtype != NVSM_U16 && dtype != NVSM_F32) return fail(ctx, NVSM_ERR_INVALID_ARG, "bad dtype");
    BurstIn bi;
    bi.frames = frames; bi.F = F; bi.H = H; bi.W = W; bi.pitch = row_pitch;
    DevicePlan *dp;
    BurstTable bt;
    Sizes z;
    nvsm_status s = prepare_call(ctx, p, bi, &dp, &bt, &z);
    if (s != NVSM_OK) return s;
    if (!workspace || workspace_bytes < ws_acc(z)) return fail(ctx, NVSM_ERR_WORKSPACE, "workspace too small for accumulate");
    hipError_t e = run_accumulate(ctx, dp, p, bt, z, dtype, power, mean_spec, mu, bispec, (char *)workspace,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "accumulate launch");
    return NVSM_OK;
}

nvsm_status nvsm_solve(nvsm_context *ctx, const nvsm_params *p, int64_t patches, const float *power,
                       const float *mean_spec, const float *bispec, const double *stf, double *amp,
                       double *phasor, void *workspace, size_t workspace_bytes, void *stream) {
    (void)workspace;
    (void)workspace_bytes;
    if (!ctx) return NVSM_ERR_INVALID_ARG;
    std::string msg;
    nvsm_status s = check_params(p, &msg);
    if (s != NVSM_OK) return fail(ctx, s, msg);
    if (patches < 0 || patches > (1 << 24)) return fail(ctx, NVSM_ERR_SHAPE, "bad patch count");
    if (!power || !mean_spec || !bispec || !stf || !amp || !phasor) return fail(ctx, NVSM_ERR_INVALID_ARG, "null buffer");
    DevicePlan *dp;
    if ((s = get_plan(ctx, p, &dp)) != NVSM_OK) return s;
    BurstTable bt;
    bt.nb = 1;
    bt.patches = (int)patches;
    bt.b[0].stf = stf;
    hipError_t e = run_solve(ctx, dp, p, bt, power, mean_spec, bispec, amp, phasor, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "solve launch");
    return NVSM_OK;
}

nvsm_status nvsm_synthesize(nvsm_context *ctx, const nvsm_params *p, int32_t H, int32_t W, const double *amp,
                            const double *phasor, const float *mu, float *patches_out, float *out,
                            void *workspace, size_t workspace_bytes, void *stream) {
    if (!ctx) return NVSM_ERR_INVALID_ARG;
    if (!amp || !phasor || !mu || !out) return fail(ctx, NVSM_ERR_INVALID_ARG, "null buffer");
    BurstIn bi;
    bi.F = 1; bi.H = H; bi.W = W; bi.pitch = W; bi.out = out;
    DevicePlan *dp;
    BurstTable bt;
    Sizes z;
    nvsm_status s = prepare_call(ctx, p, bi, &dp, &bt, &z);
    if (s != NVSM_OK) return s;
    float *pb = patches_out;
    if (!pb) {
        if (!workspace || workspace_bytes < z.patches) return fail(ctx, NVSM_ERR_WORKSPACE, "workspace too small for synthesize");
        pb = (float *)workspace;
    }
    hipError_t e = run_synth(ctx, dp, p, bt, amp, phasor, mu, pb, true, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "synthesize launch");
    return NVSM_OK;
}

nvsm_status nvsm_reconstruct(nvsm_context *ctx, const nvsm_params *p, const void *frames, nvsm_dtype dtype,
                             int32_t F, int32_t H, int32_t W, int64_t row_pitch, const double *stf, float *out,
                             void *workspace, size_t workspace_bytes, void *stream) {
    if (!ctx) return NVSM_ERR_INVALID_ARG;
    if (!frames || !stf || !out) return fail(ctx, NVSM_ERR_INVALID_ARG, "null buffer");
    if (dtype != NVSM_U16 && dtype != NVSM_F32) return fail(ctx, NVSM_ERR_INVALID_ARG, "bad dtype");
    BurstIn bi;
    bi.frames = frames; bi.F = F; bi.H = H; bi.W = W; bi.pitch = row_pitch; bi.stf = stf; bi.out = out;
    DevicePlan *dp;
    BurstTable bt;
    Sizes z;
    nvsm_status s = prepare_call(ctx, p, bi, &dp, &bt, &z);
    if (s != NVSM_OK) return s;
    if (!workspace || workspace_bytes < ws_rec(z)) return fail(ctx, NVSM_ERR_WORKSPACE, "workspace too small for reconstruct");
    hipError_t e = run_reconstruct(ctx, dp, p, bt, z, dtype, (char *)workspace, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "reconstruct launch");
    return NVSM_OK;
}

nvsm_status nvsm_reconstruct_noalloc(nvsm_context *ctx, const nvsm_params *p, const void *frames, nvsm_dtype dtype,
                                     int32_t F, int32_t H, int32_t W, int64_t row_pitch, const double *stf,
                                     float *out, void *stream) {
    if (!ctx) return NVSM_ERR_INVALID_ARG;
    if (!frames || !stf || !out) return fail(ctx, NVSM_ERR_INVALID_ARG, "null buffer");
    if (dtype != NVSM_U16 && dtype != NVSM_F32) return fail(ctx, NVSM_ERR_INVALID_ARG, "bad dtype");
    std::string msg;
    nvsm_status s = check_params(p, &msg);
    if (s != NVSM_OK) return fail(ctx, s, msg);
    BurstIn bi;
    bi.frames = frames; bi.F = F; bi.H = H; bi.W = W; bi.pitch = row_pitch; bi.stf = stf; bi.out = out;
    if ((s = check_burst(p, bi, &msg)) != NVSM_OK) return fail(ctx, s, msg);
    DevicePlan *dp = find_plan(ctx, p);
    if (!dp)
        return fail(ctx, NVSM_ERR_INVALID_ARG,
                    "no tables for these parameters: call nvsm_prepare (or any compute call) with them first");
    void *scr = scratch_address(ctx->device);
    if (!scr) return fail(ctx, NVSM_ERR_HIP, "scratch array not set up on this device");
    BurstTable bt;
    int64_t rec;
    Sizes z;
    make_table(p, &bi, 1, &bt, &rec);
    sizes_for(p->patch, bt, rec, (int64_t)(dp->h.W.size() / 2), dp->h.s_count, &z, p->noise_bias == 2);
    if (ws_rec(z) > SCRATCH_BYTES)
        return fail(ctx, NVSM_ERR_WORKSPACE,
                    "burst needs " + std::to_string(ws_rec(z)) + " bytes of workspace, more than the " +
                        std::to_string(SCRATCH_BYTES) + "-byte scratch array: use nvsm_reconstruct");
    // no stage events here (creating one may allocate)
    const bool prof = ctx->prof;
    ctx->prof = false;
    hipError_t e = run_reconstruct(ctx, dp, p, bt, z, dtype, (char *)scr, (hipStream_t)stream);
    ctx->prof = prof;
    if (e != hipSuccess) return hip_fail(ctx, e, "reconstruct launch");
    return NVSM_OK;
}

// Splits the bursts, in order, into launch groups of at most MAX_BURSTS
// whose workspace fits in cap bytes (a group of one burst always forms).
static void batch_groups(const nvsm_params *p, const BurstIn *bi, int n, int64_t nW, int64_t S, size_t cap,
                         std::vector<std::pair<int, int>> *groups, size_t *largest) {
    groups->clear();
    *largest = 0;
    int i = 0;
    while (i < n) {
        int j = i + 1;
        BurstTable bt;
        int64_t rec;
        Sizes z;
        make_table(p, bi + i, 1, &bt, &rec);
        sizes_for(p->patch, bt, rec, nW, S, &z, p->noise_bias == 2);
        size_t need = ws_rec(z);
        while (j < n && j - i < MAX_BURSTS) {
            make_table(p, bi + i, j + 1 - i, &bt, &rec);
            sizes_for(p->patch, bt, rec, nW, S, &z, p->noise_bias == 2);
            if (ws_rec(z) > cap) break;
            need = ws_rec(z);
            ++j;
        }
        *largest = std::max(*largest, need);
        groups->push_back({i, j});
        i = j;
    }
}

static nvsm_status read_bursts(const nvsm_params *p, const nvsm_burst *bursts, int32_t n, bool need_ptrs,
                               std::vector<BurstIn> *bi, std::string *msg) {
    if (!bursts || n < 1) { *msg = "no bursts"; return NVSM_ERR_INVALID_ARG; }
    bi->resize(n);
    for (int i = 0; i < n; ++i) {
        BurstIn &b = (*bi)[i];
        b.frames = bursts[i].frames; b.F = bursts[i].F; b.H = bursts[i].H; b.W = bursts[i].W;
        b.pitch = bursts[i].row_pitch; b.stf = bursts[i].stf; b.out = bursts[i].out;
        if (need_ptrs && (!b.frames || !b.stf || !b.out)) { *msg = "null buffer in burst " + std::to_string(i); return NVSM_ERR_INVALID_ARG; }
        nvsm_status s = check_burst(p, b, msg);
        if (s != NVSM_OK) { *msg += " (burst " + std::to_string(i) + ")"; return s; }
    }
    return NVSM_OK;
}

nvsm_status nvsm_batch_plan(const nvsm_params *p, const nvsm_burst *bursts, int32_t n, size_t *ws_min,
                            size_t *ws_all) {
    std::string msg;
    if (!ws_min || !ws_all) return NVSM_ERR_INVALID_ARG;
    nvsm_status s = check_params(p, &msg);
    if (s != NVSM_OK) return s;
    std::vector<BurstIn> bi;
    if ((s = read_bursts(p, bursts, n, false, &bi, &msg)) != NVSM_OK) return s;
    int64_t nW, S;
    int shells;
    try {
        count_sets(p, &nW, &S, &shells);
    } catch (const std::bad_alloc &) {
        return NVSM_ERR_OOM;
    }
    std::vector<std::pair<int, int>> g;
    size_t largest;
    batch_groups(p, bi.data(), n, nW, S, 0, &g, &largest);          // one burst per group
    *ws_min = largest;
    batch_groups(p, bi.data(), n, nW, S, SIZE_MAX, &g, &largest);   // groups of MAX_BURSTS
    *ws_all = largest;
    return NVSM_OK;
}

nvsm_status nvsm_reconstruct_batch(nvsm_context *ctx, const nvsm_params *p, nvsm_dtype dtype,
                                   const nvsm_burst *bursts, int32_t n, void *workspace, size_t workspace_bytes,
                                   void *stream) {
    if (!ctx) return NVSM_ERR_INVALID_ARG;
    if (dtype != NVSM_U16 && dtype != NVSM_F32) return fail(ctx, NVSM_ERR_INVALID_ARG, "bad dtype");
    std::string msg;
    nvsm_status s = check_params(p, &msg);
    if (s != NVSM_OK) return fail(ctx, s, msg);
    std::vector<BurstIn> bi;
    if ((s = read_bursts(p, bursts, n, true, &bi, &msg)) != NVSM_OK) return fail(ctx, s, msg);
    DevicePlan *dp;
    if ((s = get_plan(ctx, p, &dp)) != NVSM_OK) return s;
    const int64_t nW = (int64_t)(dp->h.W.size() / 2), S = dp->h.s_count;
    std::vector<std::pair<int, int>> groups;
    size_t largest;
    batch_groups(p, bi.data(), n, nW, S, workspace_bytes, &groups, &largest);
    if (!workspace || workspace_bytes < largest) return fail(ctx, NVSM_ERR_WORKSPACE, "workspace too small for the largest burst");
    for (auto &g : groups) {
        BurstTable bt;
        int64_t rec;
        Sizes z;
        make_table(p, bi.data() + g.first, g.second - g.first, &bt, &rec);
        sizes_for(p->patch, bt, rec, nW, S, &z, p->noise_bias == 2);
        hipError_t e = run_reconstruct(ctx, dp, p, bt, z, dtype, (char *)workspace, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "batch launch");
    }
    return NVSM_OK;
}

nvsm_status nvsm_autotune(nvsm_context *ctx, const nvsm_params *p, const void *frames, nvsm_dtype dtype,
                          int32_t F, int32_t H, int32_t W, int64_t row_pitch, void *workspace,
                          size_t workspace_bytes, void *stream, int32_t *slots_out, int32_t *form_out) {
    if (!ctx) return NVSM_ERR_INVALID_ARG;
    if (!frames) return fail(ctx, NVSM_ERR_INVALID_ARG, "null buffer");
    if (dtype != NVSM_U16 && dtype != NVSM_F32) return fail(ctx, NVSM_ERR_INVALID_ARG, "bad dtype");
    BurstIn bi;
    bi.frames = frames; bi.F = F; bi.H = H; bi.W = W; bi.pitch = row_pitch;
    DevicePlan *dp;
    BurstTable bt;
    Sizes z;
    nvsm_status s = prepare_call(ctx, p, bi, &dp, &bt, &z);
    if (s != NVSM_OK) return s;
    if (!workspace || workspace_bytes < ws_rec(z)) return fail(ctx, NVSM_ERR_WORKSPACE, "workspace too small for autotune");
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)workspace;
    float *power = (float *)w; w += z.power;
    float *mean = (float *)w; w += z.mean;
    float *mu = (float *)w; w += z.mu;
    float *bis = (float *)w; w += z.bispec;
    w += z.amp + z.phasor + z.patches;
    const bool prof = ctx->prof;
    ctx->prof = false;
    // spectra once; the candidates only differ in the bispectrum launch
    hipError_t e = run_accumulate(ctx, dp, p, bt, z, dtype, power, mean, mu, nullptr, w, st);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = 1e30f;
    std::pair<int, int> pick(16, 0);
    const int cand[4][2] = {{16, 0}, {16, 1}, {24, 0}, {24, 1}};
    for (int c = 0; c < 4 && e == hipSuccess; ++c) {
        DevicePlan *dc;
        if ((s = get_plan(ctx, p, cand[c][0], &dc)) != NVSM_OK) break;
        BispecArgs b;
        b.N = p->patch; b.bt = bt; b.spectra = (const float2 *)w;
        b.n_items = dc->h.n_items; b.slots = dc->h.slots; b.items = dc->items; b.group_xy = dc->group_xy;
        b.slot_v = dc->slot; b.out_idx = dc->out_idx; b.bispec = (float2 *)bis; b.s_count = z.S;
        b.form = cand[c][1]; b.queue = queue_of(w, z);
        float t = 1e30f;
        for (int r = 0; r < 3 && e == hipSuccess; ++r) {       // the first run warms up
            e = hipEventRecord(e0, st);
            if (e == hipSuccess) e = launch_bispec(b, st);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (r > 0) t = std::min(t, ms);
        }
        if (e == hipSuccess && t < best) { best = t; pick = std::make_pair(cand[c][0], cand[c][1]); }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    ctx->prof = prof;
    if (s != NVSM_OK) return s;
    if (e != hipSuccess) return hip_fail(ctx, e, "autotune");
    ctx->tuned[std::make_tuple(p->patch, p->u_cut, p->v_radius)] = pick;
    if (slots_out) *slots_out = pick.first;
    if (form_out) *form_out = pick.second;
    return NVSM_OK;
}

// The central crop the v-radius tuner works on: at most TUNE_CROP px a side,
// x0 a multiple of 4 (keeps vector pixel loads).
constexpr int TUNE_CROP = 512;
static void tune_crop(int H, int W, int *y0, int *x0, int *Hc, int *Wc) {
    *Hc = std::min(H, TUNE_CROP);
    *Wc = std::min(W, TUNE_CROP);
    *y0 = (H - *Hc) / 2;
    *x0 = (W - *Wc) / 2 / 4 * 4;
}

static nvsm_status tune_sizes(const nvsm_params *p, int32_t H, int32_t W, int32_t F, int32_t r_max, Sizes *z,
                              std::string *msg) {
    nvsm_params q = *p;
    q.v_radius = r_max;
    nvsm_status s = check_params(&q, msg);
    if (s != NVSM_OK) return s;
    if ((s = check_shape(&q, H, W, F, msg)) != NVSM_OK) return s;
    int y0, x0, Hc, Wc;
    tune_crop(H, W, &y0, &x0, &Hc, &Wc);
    int64_t nW, S;
    int shells;
    try {
        count_sets(&q, &nW, &S, &shells);
    } catch (const std::bad_alloc &) {
        return NVSM_ERR_OOM;
    }
    BurstIn bi;
    bi.F = F; bi.H = Hc; bi.W = Wc; bi.pitch = Wc;
    BurstTable bt;
    int64_t rec;
    make_table(&q, &bi, 1, &bt, &rec);
    sizes_for(q.patch, bt, rec, nW, S, z, q.noise_bias == 2);
    return NVSM_OK;
}

nvsm_status nvsm_tune_radius_plan(const nvsm_params *p, int32_t H, int32_t W, int32_t F, int32_t r_max,
                                  size_t *ws_bytes) {
    if (!ws_bytes) return NVSM_ERR_INVALID_ARG;
    std::string msg;
    Sizes z;
    nvsm_status s = tune_sizes(p, H, W, F, r_max, &z, &msg);
    if (s != NVSM_OK) return s;
    *ws_bytes = ws_rec(z);
    return NVSM_OK;
}

nvsm_status nvsm_tune_radius(nvsm_context *ctx, const nvsm_params *p, const void *frames, nvsm_dtype dtype,
                             int32_t F, int32_t H, int32_t W, int64_t row_pitch, const double *stf, int32_t r_min,
                             int32_t r_max, double tol, void *workspace, size_t workspace_bytes, void *stream,
                             int32_t *r_out, double *err) {
    if (!ctx) return NVSM_ERR_INVALID_ARG;
    if (!frames || !stf || !r_out) return fail(ctx, NVSM_ERR_INVALID_ARG, "null buffer");
    if (dtype != NVSM_U16 && dtype != NVSM_F32) return fail(ctx, NVSM_ERR_INVALID_ARG, "bad dtype");
    if (r_min < 1 || r_min > r_max) return fail(ctx, NVSM_ERR_INVALID_ARG, "need 1 <= r_min <= r_max");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(ctx, NVSM_ERR_INVALID_ARG, "tol must be finite and >= 0");
    std::string msg;
    Sizes zmax;
    nvsm_status s = tune_sizes(p, H, W, F, r_max, &zmax, &msg);
    if (s != NVSM_OK) return fail(ctx, s, msg);
    {
        nvsm_params q = *p;
        q.v_radius = r_min;
        if ((s = check_params(&q, &msg)) != NVSM_OK) return fail(ctx, s, msg);
    }
    BurstIn full;
    full.frames = frames; full.F = F; full.H = H; full.W = W; full.pitch = row_pitch; full.stf = stf;
    if ((s = check_burst(p, full, &msg)) != NVSM_OK) return fail(ctx, s, msg);
    if (!workspace || workspace_bytes < ws_rec(zmax)) return fail(ctx, NVSM_ERR_WORKSPACE, "workspace too small for tuning");
    int y0, x0, Hc, Wc;
    tune_crop(H, W, &y0, &x0, &Hc, &Wc);
    const size_t px = dtype == NVSM_F32 ? 4 : 2;
    BurstIn bi = full;
    bi.frames = (const char *)frames + ((size_t)y0 * row_pitch + x0) * px;
    bi.H = Hc; bi.W = Wc;
    hipStream_t st = (hipStream_t)stream;
    const bool prof = ctx->prof;
    ctx->prof = false;
    // phasors of the crop's patches at radius r (and the weights: the mean
    // power at each w of W), on the host
    auto run = [&](int r, std::vector<double> *wt, std::vector<double> *ph) -> nvsm_status {
        nvsm_params q = *p;
        q.v_radius = r;
        q.phase_method = 0;
        DevicePlan *dp;
        BurstTable bt;
        Sizes z;
        nvsm_status t = prepare_call(ctx, &q, bi, &dp, &bt, &z);
        if (t != NVSM_OK) return t;
        char *w = (char *)workspace;
        float *power = (float *)w; w += z.power;
        float *mean = (float *)w; w += z.mean;
        float *mu = (float *)w; w += z.mu;
        float *bis = (float *)w; w += z.bispec;
        double *a = (double *)w; w += z.amp;
        double *e = (double *)w; w += z.phasor;
        w += z.patches;
        hipError_t h = run_accumulate(ctx, dp, &q, bt, z, dtype, power, mean, mu, bis, w, st);
        if (h == hipSuccess) h = run_solve(ctx, dp, &q, bt, power, mean, bis, a, e, st);
        const int N = q.patch;
        std::vector<float> pw;
        if (wt) pw.resize((size_t)z.P * N * N);
        ph->resize((size_t)z.P * z.nW * 2);
        if (h == hipSuccess) h = hipMemcpyAsync(ph->data(), e, ph->size() * 8, hipMemcpyDeviceToHost, st);
        if (h == hipSuccess && wt) h = hipMemcpyAsync(pw.data(), power, pw.size() * 4, hipMemcpyDeviceToHost, st);
        if (h == hipSuccess) h = hipStreamSynchronize(st);
        if (h != hipSuccess) return hip_fail(ctx, h, "radius tuning");
        if (wt) {
            // weight: the mean power above the patch's noise floor (the mean
            // power where |u| > N/2 + 2, the level noise_bias 1 removes), so
            // that frequencies at the floor, whose phases carry no signal,
            // do not count
            wt->resize((size_t)z.P * z.nW);
            const std::vector<int32_t> &Wl = dp->h.W;
            const double lim = (N / 2 + 2.0) * (N / 2 + 2.0);
            for (int64_t k = 0; k < z.P; ++k) {
                const float *pk = pw.data() + (size_t)k * N * N;
                double acc = 0.0;
                int64_t cnt = 0;
                for (int j = 0; j < N * N; ++j) {
                    int ux = j % N, uy = j / N;
                    ux = ux >= N / 2 ? ux - N : ux;
                    uy = uy >= N / 2 ? uy - N : uy;
                    if ((double)(ux * ux + uy * uy) > lim) { acc += pk[j]; ++cnt; }
                }
                const double floor_k = cnt ? acc / (double)cnt : 0.0;
                for (int64_t i = 0; i < z.nW; ++i) {
                    const double pwi = pk[(size_t)(Wl[2 * i + 1] & (N - 1)) * N + (Wl[2 * i] & (N - 1))];
                    (*wt)[k * z.nW + i] = std::max(pwi - floor_k, 0.0);
                }
            }
        }
        return NVSM_OK;
    };
    std::vector<double> wmax, emax, e;
    s = run(r_max, &wmax, &emax);
    if (s == NVSM_OK && err)
        for (int r = r_min; r <= r_max; ++r) err[r - r_min] = std::nan("");
    int pick = r_max;
    for (int r = r_min; s == NVSM_OK && r <= r_max; ++r) {
        double d = 0.0;
        if (r < r_max) {
            if ((s = run(r, nullptr, &e)) != NVSM_OK) break;
            double num = 0.0, den = 0.0;
            for (size_t i = 0; i < wmax.size(); ++i) {
                // wrapped phase difference: arg(e conj emax)
                const double re = e[2 * i] * emax[2 * i] + e[2 * i + 1] * emax[2 * i + 1];
                const double im = e[2 * i + 1] * emax[2 * i] - e[2 * i] * emax[2 * i + 1];
                const double dphi = std::atan2(im, re);
                num += wmax[i] * dphi * dphi;
                den += wmax[i];
            }
            d = den > 0.0 ? std::sqrt(num / den) : 0.0;
        }
        if (err) err[r - r_min] = d;
        if (d <= tol) { pick = r; break; }
    }
    ctx->prof = prof;
    if (s != NVSM_OK) return s;
    *r_out = pick;
    return NVSM_OK;
}

nvsm_status nvsm_set_launch(nvsm_context *ctx, const nvsm_params *p, int32_t slots, int32_t form) {
    if (!ctx) return NVSM_ERR_INVALID_ARG;
    std::string msg;
    nvsm_status s = check_params(p, &msg);
    if (s != NVSM_OK) return fail(ctx, s, msg);
    if ((slots != 16 && slots != 24) || (form != 0 && form != 1))
        return fail(ctx, NVSM_ERR_INVALID_ARG, "slots must be 16 or 24 and form 0 or 1");
    ctx->tuned[std::make_tuple(p->patch, p->u_cut, p->v_radius)] = std::make_pair((int)slots, (int)form);
    DevicePlan *dp;
    return get_plan(ctx, p, &dp);
}

nvsm_status nvsm_stream_plan(const nvsm_params *p, int32_t H, int32_t W, int32_t group_frames,
                             size_t *state_bytes, size_t *ws_bytes) {
    std::string msg;
    if (!state_bytes || !ws_bytes) return NVSM_ERR_INVALID_ARG;
    nvsm_status s = check_params(p, &msg);
    if (s != NVSM_OK) return s;
    if ((s = check_shape(p, H, W, group_frames, &msg)) != NVSM_OK) return s;
    HostPlan h;
    try {
        if (!build_plan(p->patch, p->u_cut, p->v_radius, STREAM_SLOTS, &h, &msg)) return NVSM_ERR_INVALID_ARG;
    } catch (const std::bad_alloc &) {
        return NVSM_ERR_OOM;
    }
    const int64_t lane_terms = (int64_t)h.n_items * BS_WAVES * STREAM_SLOTS * 64;
    BurstIn bi;
    bi.F = group_frames; bi.H = H; bi.W = W; bi.pitch = W;
    BurstTable bt;
    int64_t rec;
    make_table(p, &bi, 1, &bt, &rec);
    Sizes z;
    sizes_for(p->patch, bt, rec, (int64_t)h.W.size() / 2, h.s_count, &z, p->noise_bias == 2);
    StreamSizes ss;
    stream_sizes(p->patch, bt.patches, (int64_t)h.W.size() / 2, h.s_count, lane_terms, ws_acc(z), &ss,
                 p->noise_bias == 2);
    *state_bytes = ss.state();
    *ws_bytes = ss.ws();
    return NVSM_OK;
}

static nvsm_status stream_prep(nvsm_context *ctx, const nvsm_params *p, int32_t H, int32_t W, int32_t G,
                               DevicePlan **dp, BurstTable *bt, Sizes *z, StreamSizes *ss) {
    std::string msg;
    nvsm_status s = check_params(p, &msg);
    if (s != NVSM_OK) return fail(ctx, s, msg);
    if ((s = check_shape(p, H, W, G, &msg)) != NVSM_OK) return fail(ctx, s, msg);
    if ((s = get_plan(ctx, p, STREAM_SLOTS, dp)) != NVSM_OK) return s;
    BurstIn bi;
    bi.F = G; bi.H = H; bi.W = W; bi.pitch = W;
    int64_t rec;
    make_table(p, &bi, 1, bt, &rec);
    sizes_for(p->patch, *bt, rec, (int64_t)((*dp)->h.W.size() / 2), (*dp)->h.s_count, z, p->noise_bias == 2);
    const int64_t lane_terms = (int64_t)(*dp)->h.n_items * BS_WAVES * (*dp)->h.slots * 64;
    stream_sizes(p->patch, bt->patches, (int64_t)((*dp)->h.W.size() / 2), (*dp)->h.s_count, lane_terms, ws_acc(*z),
                 ss, p->noise_bias == 2);
    return NVSM_OK;
}

nvsm_status nvsm_stream_add(nvsm_context *ctx, const nvsm_params *p, const void *frames, nvsm_dtype dtype,
                            int32_t G, int32_t H, int32_t W, int64_t row_pitch, int32_t frames_before,
                            int32_t total_frames, void *state, size_t state_bytes, void *ws, size_t ws_bytes,
                            void *stream) {
    if (!ctx) return NVSM_ERR_INVALID_ARG;
    if (!frames) return fail(ctx, NVSM_ERR_INVALID_ARG, "null buffer");
    if (dtype != NVSM_U16 && dtype != NVSM_F32) return fail(ctx, NVSM_ERR_INVALID_ARG, "bad dtype");
    if (frames_before < 0) return fail(ctx, NVSM_ERR_INVALID_ARG, "frames_before < 0");
    if (total_frames != 0 && total_frames != frames_before + G)
        return fail(ctx, NVSM_ERR_INVALID_ARG, "total_frames must be 0 or frames_before + G");
    DevicePlan *dp;
    BurstTable bt;
    Sizes z;
    StreamSizes ss;
    nvsm_status s = stream_prep(ctx, p, H, W, G, &dp, &bt, &z, &ss);
    if (s != NVSM_OK) return s;
    BurstIn bi;
    bi.frames = frames; bi.F = G; bi.H = H; bi.W = W; bi.pitch = row_pitch;
    std::string msg;
    if ((s = check_burst(p, bi, &msg)) != NVSM_OK) return fail(ctx, s, msg);
    bt.b[0].frames = frames;
    bt.b[0].pitch = row_pitch;
    if (!state || state_bytes < ss.state()) return fail(ctx, NVSM_ERR_WORKSPACE, "stream state too small");
    if (!ws || ws_bytes < ss.ws()) return fail(ctx, NVSM_ERR_WORKSPACE, "stream workspace too small");
    StreamView v = stream_view((char *)state, (char *)ws, ss);
    const int mode = total_frames ? 2 : 1;
    const int first = frames_before == 0;
    const float inv_total = total_frames ? 1.0f / (float)total_frames : 0.f;
    hipStream_t st = (hipStream_t)stream;
    char *gw = v.group;
    IngestArgs a;
    a.N = p->patch;
    a.f32 = dtype == NVSM_F32;
    a.bt = bt;
    a.stride = p->stride;
    a.chunk_frames = CHUNK_FRAMES; a.window = p->window;
    a.vec = vec_ok(p, bt, a.f32 ? 4 : 2);
    a.inv_wsum = (float)(1.0 / (p->window ? dp->h.hann_sum2 : (double)p->patch * p->patch));
    a.twiddle = dp->twiddle; a.hann = dp->hann;
    a.spectra = (float2 *)gw;
    a.ppart = (float *)(gw + z.spectra);
    a.mpart = (float *)(gw + z.spectra + z.ppart);
    a.mupart = (float *)(gw + z.spectra + z.ppart + z.mpart);
    a.power = v.power; a.mean_spec = v.mean; a.mu = v.mu;
    a.stream_mode = mode; a.stream_first = first;
    a.psc = v.psc; a.msc = v.msc; a.musc = v.musc; a.inv_total = inv_total;
    hipError_t e;
    NoiseArgs na;
    if (p->noise_bias == 2) {
        // the group's photon-noise sums go into the state's running sums;
        // the last group writes their means where the bispectrum launch
        // reads them (the layout of the accumulate scratch)
        char *q = gw + z.spectra + z.ppart + z.mpart + z.mupart;
        na.in = a;
        na.inv_gain = (float)(1.0 / p->photons_per_adu);
        na.cpart = (float2 *)q; q += z.cpart;
        na.spart = (float *)q; q += z.spart;
        na.cgrid = (float2 *)q; q += z.cw;
        na.nbar = (float *)q;
        na.csc = v.csc; na.ssc = v.ssc;
    }
    {
        StageTimer t(ctx, ST_INGEST, st);
        e = launch_ingest(a, st);
        if (e == hipSuccess && p->noise_bias == 2) e = launch_noise(na, st);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "stream ingest");
    BispecArgs b;
    b.N = p->patch; b.bt = bt; b.spectra = a.spectra;
    b.n_items = dp->h.n_items; b.slots = dp->h.slots; b.items = dp->items; b.group_xy = dp->group_xy;
    b.slot_v = dp->slot; b.out_idx = dp->out_idx;
    b.bispec = v.bis; b.s_count = z.S;
    b.form = choice_of(ctx, p).second; b.queue = queue_of(gw, z);
    b.acc.sum = v.acc_s; b.acc.comp = v.acc_c; b.acc.mode = mode; b.acc.first = first;
    b.acc.n_items = dp->h.n_items; b.acc.inv_total = inv_total;
    if (p->noise_bias == 2 && mode == 2) {
        b.acc.noise_c = na.cgrid;
        b.acc.noise_t = na.nbar;
    }
    {
        StageTimer t(ctx, ST_BISPEC, st);
        e = launch_bispec(b, st);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "stream bispectrum");
    return NVSM_OK;
}

nvsm_status nvsm_stream_finish(nvsm_context *ctx, const nvsm_params *p, int32_t H, int32_t W, const double *stf,
                               float *out, void *ws, size_t ws_bytes, void *stream) {
    if (!ctx) return NVSM_ERR_INVALID_ARG;
    if (!stf || !out) return fail(ctx, NVSM_ERR_INVALID_ARG, "null buffer");
    DevicePlan *dp;
    BurstTable bt;
    Sizes z;
    StreamSizes ss;
    nvsm_status s = stream_prep(ctx, p, H, W, 1, &dp, &bt, &z, &ss);
    if (s != NVSM_OK) return s;
    const size_t final_bytes = ss.ws() - ss.group;
    if (!ws || ws_bytes < final_bytes) return fail(ctx, NVSM_ERR_WORKSPACE, "stream workspace too small");
    bt.b[0].stf = stf;
    bt.b[0].out = out;
    StreamView v = stream_view(nullptr, (char *)ws, ss);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = run_solve(ctx, dp, p, bt, v.power, v.mean, (const float *)v.bis, v.amp, v.phasor, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "stream solve");
    e = run_synth(ctx, dp, p, bt, v.amp, v.phasor, v.mu, v.patches, true, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "stream synthesize");
    return NVSM_OK;
}

// sqrt(0.023) r0^(-5/6) N^(5/6) with r0 = (N/2) / (D/r0) px (see k_stf.hip)
static float screen_amp(int N, double d_over_r0) {
    const double r0 = (N / 2.0) / d_over_r0;
    return (float)(std::sqrt(0.023) * std::pow(r0, -5.0 / 6.0) * std::pow((double)N, 5.0 / 6.0));
}

static nvsm_status stf_sizes(const nvsm_params *p, int32_t screens, int *pairs, int *nwg, size_t *part_a,
                             size_t *part_s, std::string *msg) {
    nvsm_status s = check_params(p, msg);
    if (s != NVSM_OK) return s;
    if (screens < 2 || screens > (1 << 24) || screens % 2) {
        *msg = "screens must be even and in [2, 2^24]";
        return NVSM_ERR_INVALID_ARG;
    }
    *pairs = screens / 2;
    *nwg = std::min(*pairs, 256);                // one workgroup per CU (the tile fills LDS)
    const size_t np = (size_t)(p->patch / 2 + 1) * p->patch;
    *part_a = align_up((size_t)*nwg * np * 8);
    *part_s = align_up((size_t)*nwg * np * 4);
    return NVSM_OK;
}

nvsm_status nvsm_model_stf_plan(const nvsm_params *p, int32_t screens, size_t *ws_bytes) {
    if (!ws_bytes) return NVSM_ERR_INVALID_ARG;
    std::string msg;
    int pairs, nwg;
    size_t pa, ps;
    nvsm_status s = stf_sizes(p, screens, &pairs, &nwg, &pa, &ps, &msg);
    if (s != NVSM_OK) return s;
    *ws_bytes = pa + ps;
    return NVSM_OK;
}

nvsm_status nvsm_model_stf(nvsm_context *ctx, const nvsm_params *p, double d_over_r0, int32_t screens,
                           uint64_t seed, double *stf, double *mean_otf, void *workspace, size_t workspace_bytes,
                           void *stream) {
    if (!ctx) return NVSM_ERR_INVALID_ARG;
    if (!stf) return fail(ctx, NVSM_ERR_INVALID_ARG, "null buffer");
    std::string msg;
    int pairs, nwg;
    size_t pa, ps;
    nvsm_status s = stf_sizes(p, screens, &pairs, &nwg, &pa, &ps, &msg);
    if (s != NVSM_OK) return fail(ctx, s, msg);
    if (!(d_over_r0 > 0.0 && d_over_r0 <= 1000.0))
        return fail(ctx, NVSM_ERR_INVALID_ARG, "d_over_r0 must be in (0, 1000]");
    if (!workspace || workspace_bytes < pa + ps) return fail(ctx, NVSM_ERR_WORKSPACE, "workspace too small");
    DevicePlan *dp;
    if ((s = get_plan(ctx, p, &dp)) != NVSM_OK) return s;
    const int N = p->patch;
    StfArgs a;
    a.N = N; a.pairs = pairs; a.nwg = nwg;
    a.amp = screen_amp(N, d_over_r0);
    a.k0 = (uint32_t)(seed & 0xffffffffu); a.k1 = (uint32_t)(seed >> 32); a.stream = 0;
    a.twiddle = dp->twiddle;
    a.part_a = (float2 *)workspace;
    a.part_s = (float *)((char *)workspace + pa);
    a.stf = stf; a.mean_otf = (double2 *)mean_otf;
    hipError_t e = launch_stf(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "model stf");
    return NVSM_OK;
}

nvsm_status nvsm_seeing_default_params(nvsm_seeing_params *out) {
    if (!out) return NVSM_ERR_INVALID_ARG;
    out->screens = 1000;
    out->points = 40;
    out->d_over_r0_min = 2.0;
    out->d_over_r0_max = 50.0;
    out->bins = 12;
    out->reserved = 0;
    out->seed = 1;
    return NVSM_OK;
}

namespace {

struct SeeingSizes {
    int cubes = 0, nx = 0, nchunks = 0, box = 0, pairs = 0, nwg = 0;
    size_t part_a = 0, part_s = 0, tab_s = 0, tab_a = 0, ratio = 0;
    size_t total() const { return part_a + part_s + tab_s + tab_a + ratio; }
};

nvsm_status seeing_sizes(const nvsm_params *p, const nvsm_seeing_params *sp, int32_t H, int32_t W, int32_t F,
                         SeeingSizes *z, std::string *msg) {
    if (!sp) { *msg = "seeing params is NULL"; return NVSM_ERR_INVALID_ARG; }
    nvsm_status s = stf_sizes(p, sp->screens, &z->pairs, &z->nwg, &z->part_a, &z->part_s, msg);
    if (s != NVSM_OK) return s;
    const int N = p->patch;
    if (sp->points < 3 || sp->points > RATIO_MAX_POINTS) { *msg = "points must be in [3, 256]"; return NVSM_ERR_INVALID_ARG; }
    if (!(sp->d_over_r0_min > 0.0 && sp->d_over_r0_min < sp->d_over_r0_max && sp->d_over_r0_max <= 1000.0)) {
        *msg = "need 0 < d_over_r0_min < d_over_r0_max <= 1000";
        return NVSM_ERR_INVALID_ARG;
    }
    if (sp->bins < 2 || sp->bins > std::min(RATIO_MAX_BINS, N / 4)) {
        *msg = "bins must be in [2, min(24, N/4)]";
        return NVSM_ERR_INVALID_ARG;
    }
    if (F < 2) { *msg = "the spectral ratio needs F >= 2"; return NVSM_ERR_SHAPE; }
    if (H < N || W < N) { *msg = "frames smaller than one cube"; return NVSM_ERR_SHAPE; }
    if ((int64_t)H * W > ((int64_t)1 << 31) - 1) { *msg = "frame too large"; return NVSM_ERR_SHAPE; }
    z->nx = W / N;
    z->cubes = (H / N) * z->nx;
    z->nchunks = (F + CHUNK_FRAMES - 1) / CHUNK_FRAMES;
    const int B = sp->bins + 2;
    z->box = (B + 1) * (2 * B + 1);
    z->tab_s = align_up((size_t)sp->points * N * N * 8);
    z->tab_a = align_up((size_t)sp->points * N * N * 16);
    z->ratio = align_up((size_t)z->cubes * z->nchunks * z->box * 3 * 4);
    return NVSM_OK;
}

}  // namespace

nvsm_status nvsm_seeing_plan(const nvsm_params *p, const nvsm_seeing_params *sp, int32_t H, int32_t W, int32_t F,
                             size_t *ws_bytes, int32_t *cubes) {
    if (!ws_bytes || !cubes) return NVSM_ERR_INVALID_ARG;
    std::string msg;
    SeeingSizes z;
    nvsm_status s = seeing_sizes(p, sp, H, W, F, &z, &msg);
    if (s != NVSM_OK) return s;
    *ws_bytes = z.total();
    *cubes = z.cubes;
    return NVSM_OK;
}

nvsm_status nvsm_seeing(nvsm_context *ctx, const nvsm_params *p, const nvsm_seeing_params *sp, const void *frames,
                        nvsm_dtype dtype, int32_t F, int32_t H, int32_t W, int64_t row_pitch, double *d_over_r0,
                        double *stf, double *curves, void *workspace, size_t workspace_bytes, void *stream) {
    if (!ctx) return NVSM_ERR_INVALID_ARG;
    if (!frames || !d_over_r0 || !stf) return fail(ctx, NVSM_ERR_INVALID_ARG, "null buffer");
    if (dtype != NVSM_U16 && dtype != NVSM_F32) return fail(ctx, NVSM_ERR_INVALID_ARG, "bad dtype");
    std::string msg;
    SeeingSizes z;
    nvsm_status s = seeing_sizes(p, sp, H, W, F, &z, &msg);
    if (s != NVSM_OK) return fail(ctx, s, msg);
    if (row_pitch < W) return fail(ctx, NVSM_ERR_SHAPE, "row_pitch < W");
    if (row_pitch > max_row_pitch(p->patch)) return fail(ctx, NVSM_ERR_SHAPE, "row_pitch too large (N * row_pitch must stay below 2^30)");
    if (!workspace || workspace_bytes < z.total()) return fail(ctx, NVSM_ERR_WORKSPACE, "workspace too small");
    DevicePlan *dp;
    if ((s = get_plan(ctx, p, &dp)) != NVSM_OK) return s;
    const int N = p->patch, J = sp->points;
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)workspace;
    float2 *part_a = (float2 *)w; w += z.part_a;
    float *part_s = (float *)w; w += z.part_s;
    double *tab_s = (double *)w; w += z.tab_s;
    double2 *tab_a = (double2 *)w; w += z.tab_a;
    float *ratio = (float *)w;
    // model curves' tables, model points m = 0..J-1
    StfArgs ma;
    ma.N = N; ma.pairs = z.pairs; ma.nwg = z.nwg;
    ma.k0 = (uint32_t)(sp->seed & 0xffffffffu); ma.k1 = (uint32_t)(sp->seed >> 32);
    ma.twiddle = dp->twiddle; ma.part_a = part_a; ma.part_s = part_s;
    hipError_t e = hipSuccess;
    for (int j = 0; j < J && e == hipSuccess; ++j) {
        const double x = sp->d_over_r0_min * std::pow(sp->d_over_r0_max / sp->d_over_r0_min, j / (J - 1.0));
        ma.amp = screen_amp(N, x);
        ma.stream = (uint32_t)j;
        ma.stf = tab_s + (size_t)j * N * N;
        ma.mean_otf = tab_a + (size_t)j * N * N;
        e = launch_stf(ma, st);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "seeing model");
    RatioArgs ra;
    ra.N = N; ra.f32 = dtype == NVSM_F32;
    const size_t px = ra.f32 ? 4 : 2;
    ra.vec = row_pitch % 4 == 0 && (uintptr_t)frames % (4 * px) == 0;
    ra.frames = frames; ra.F = F; ra.H = H; ra.cubes = z.cubes; ra.nx = z.nx; ra.chunk_frames = CHUNK_FRAMES;
    ra.window = p->window; ra.B = sp->bins + 2; ra.pitch = row_pitch;
    ra.inv_wsum = (float)(1.0 / (p->window ? dp->h.hann_sum2 : (double)N * N));
    ra.twiddle = dp->twiddle; ra.hann = dp->hann; ra.part = ratio;
    if ((e = launch_ratio(ra, st)) != hipSuccess) return hip_fail(ctx, e, "seeing ratio");
    SeeingFitArgs fa;
    fa.N = N; fa.cubes = z.cubes; fa.nchunks = z.nchunks; fa.F = F; fa.B = sp->bins + 2; fa.Q = sp->bins; fa.J = J;
    fa.window = p->window; fa.lo = sp->d_over_r0_min; fa.hi = sp->d_over_r0_max;
    fa.part = ratio; fa.tab_s = tab_s; fa.tab_a = tab_a; fa.x = d_over_r0; fa.curves = curves;
    if ((e = launch_seeing_fit(fa, st)) != hipSuccess) return hip_fail(ctx, e, "seeing fit");
    // the burst's model STF at the estimate (read on the device), model point m = J
    ma.amp = 0.f; ma.x_dev = d_over_r0; ma.stream = (uint32_t)J; ma.stf = stf; ma.mean_otf = nullptr;
    if ((e = launch_stf(ma, st)) != hipSuccess) return hip_fail(ctx, e, "seeing stf");
    return NVSM_OK;
}

nvsm_status nvsm_profile_enable(nvsm_context *ctx, int32_t enable) {
    if (!ctx) return NVSM_ERR_INVALID_ARG;
    ctx->prof = enable != 0;
    return NVSM_OK;
}

nvsm_status nvsm_profile_read(nvsm_context *ctx, double *ms, int64_t *count, int32_t n) {
    if (!ctx || !ms || !count || n < NSTAGE) return NVSM_ERR_INVALID_ARG;
    nvsm_status s = NVSM_OK;
    for (auto &r : ctx->recs) {
        float t = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) {
            s = fail(ctx, NVSM_ERR_HIP, "event timing failed");
        } else {
            ms[r.stage] += t;
            count[r.stage] += 1;
        }
        ctx->free_ev.push_back(r.a);
        ctx->free_ev.push_back(r.b);
    }
    ctx->recs.clear();
    return s;
}

}  // extern "C"
