// Host-side planning: index sets, the shell schedule of the phase
// recursion and the work decomposition of the bispectrum kernel.
// Pure C++ (no HIP), so it can be unit-tested on any host.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace nvsm {

// Bispectrum kernel geometry: a wave's 64 lanes hold a group of w close in
// angle and radius, its K slots hold v values shared by the whole wave.
constexpr int BS_LANES = 64;
constexpr int BS_MAX_SLOTS = 32;     // largest slot count per wave
constexpr int BS_WAVES = 4;            // waves per workgroup
// Staged region extent (pitch x height) per frame, in whole 128s: larger
// for more slots per wave, whose items span more v.  With 16 slots, 1024
// (two 16-byte loads per lane and frame) holds the full items of every
// supported (N, R); the planner would give a group whose region is larger
// items of fewer v.
constexpr int bs_max_region(int slots) { return slots <= 16 ? 1024 : 2048; }
constexpr int BS_ITEM_INTS = 12;       // ints per workgroup item

// Least-squares phase steps: segments (w) are taken in rounds of
// LSQ_ROUND; accumulators live in LDS for the inner entries (|w| <= R) and
// a ring for the rest, LSQ_ACC entries in all.
constexpr int LSQ_ROUND = 64;
// Waves of the phase-solve workgroup (one w each per unit).
constexpr int SOLVE_WAVES = 8;
// Samples per lane in a phase-solve unit: a w's samples over 64 lanes,
// rounded up to 2, 4 or 8 (the largest sample count of any w decides).
constexpr int SOLVE_MAX_SAMPLES = 512;
constexpr int solve_samples_per_lane(int max_sw) { return max_sw <= 128 ? 2 : max_sw <= 256 ? 4 : 8; }
constexpr int LSQ_ACC = 3968;

struct Tiling {
    int ny = 0, nx = 0;
    std::vector<int32_t> ys, xs;
};

// Rows k start at min(k*s, L-N), k < ceil((L-N)/s)+1 (last tile flush).
bool make_tiling(int H, int W, int N, int s, Tiling *t);

struct HostPlan {
    int N = 0, uc = 0, R = 0;
    // W in storage order as (wx, wy) pairs, and the S offset of each w.
    std::vector<int32_t> W;
    std::vector<int32_t> woff;          // |W|+1
    std::vector<int32_t> shell_wb;      // shells+1: W range of each shell
    // Phase-solve groups: runs of consecutive shells in which no sample
    // reads a w of its own run (both sides lie before the run's first w),
    // so that all w of a group can be solved at once.  group_wb: groups+1,
    // W range of each group; group 0 is the seed shell.
    std::vector<int32_t> group_wb;
    // Phasor window of the phase solve: W entries [0, n_inner) (|w| <= R)
    // stay resident; the others live in a ring of ring_size entries.  A
    // group reads ring entries >= its lowest index, so entry i sits at ring
    // slot (i - n_inner - group_ring_off[g]) reduced once by ring_size.
    int n_inner = 0, ring_size = 0;
    std::vector<int32_t> group_ring_off;  // groups: multiple of ring_size
    // phase_code with W indices replaced by the LDS slot each phasor has
    // while the sample's group is solved, and the slot of every w.
    std::vector<uint32_t> phase_slot_code;
    std::vector<int32_t> w_slot;
    // phase_slot_code as the phase-solve kernel reads it: one block of
    // solve_pad = 64 x solve_samples_per_lane(max_sw) codes per w, entry k
    // of block w the code of sample woff[w] + k for k below its count and
    // otherwise two reads of zero_slot (= n_inner + ring_size, a window
    // slot past the ring that holds a zero phasor, so that padding samples
    // add nothing); the seeds' blocks are all padding.  Empty when some w
    // has more than SOLVE_MAX_SAMPLES samples.
    int max_sw = 0, solve_pad = 0, zero_slot = 0;
    std::vector<uint32_t> solve_code;
    // Phase-solve units: each group after the first (the seeds) cut into
    // units of at most SOLVE_WAVES w, one w per wave.  solve_units[(u *
    // SOLVE_WAVES + j) * 4 + 0..3] = (w of wave j or -1, its first S index,
    // its sample count + 65536 if u is the last unit of its group, the LDS
    // slot of its phasor).  The units of one group are independent; a
    // group's results are read only by later groups.
    int n_units = 0;
    std::vector<int32_t> solve_units;
    // Least-squares rounds: before round r (segments [r, r + 1) * LSQ_ROUND)
    // the entries [n_inner, lsq_fin[r]) are targets of no later segment;
    // lsq_fin[0] = n_inner, lsq_fin[rounds] = |W|.  lsq_span is the most
    // ring entries live in one round, [lsq_fin[r], (r + 1) * LSQ_ROUND).
    std::vector<int32_t> lsq_fin;
    int lsq_span = 0;
    // Per S entry: lookup codes of (w - v) and v in the phasor table
    // (bits 0..14 index into W, bit 15 set = use the conjugate).
    std::vector<uint32_t> phase_code;
    int64_t s_count = 0;
    // Bispectrum work items.  items[g*12 + 0..11] = w group, region x0,
    // region y0, region width, region height, region points (width x
    // height), region row pitch in LDS, 0, then the slot count ns of each of
    // the BS_WAVES waves (a multiple of 4, 4 <= ns <= K).  The
    // region holds I(w - v) for every lane's w and every slot's v of the
    // item.
    int slots = 0;                      // v slots per wave (K)
    int n_items = 0;
    std::vector<int32_t> items;
    // group_xy[(group*64 + lane)*2 + 0/1] = (wx, wy) of the lane's w (idle
    // lanes repeat lane 0's w and never write a result).
    int n_groups = 0;
    std::vector<int32_t> group_xy;
    int max_region = 0;                 // largest region points of any item
    // slot[((g*BS_WAVES + wave)*K + k)*2 + 0] = vy * region_pitch + vx
    // (offset of v in the staged region), [..+1] = offset of I(v) in a
    // frame's stored spectrum record (rows -16 .. N/2-1).
    std::vector<int32_t> slot_v;
    // out_idx[((g*BS_WAVES + wave)*K + k)*64 + lane] = S index or -1
    std::vector<int32_t> out_idx;
    int64_t computed_terms = 0;         // wave slots x 64 lanes actually run
    // Constant tables.
    std::vector<float> twiddle;         // 2N: exp(-2 pi i k / N), k < N
    std::vector<float> hann;            // N: periodic Hann taper
    std::vector<float> filt;            // |W|: diffraction OTF at |w|/(N/2)
    double hann_sum2 = 0;               // sum of the 2-D taper
};

// Builds everything above; returns false with *err set on bad sizes.
bool build_plan(int N, int uc, int R, int slots, HostPlan *out, std::string *err);

// The phase solve's part of the plan for the groups in group_wb (W, woff,
// phase_code, shell_wb and R already set): the phasor window, the slot
// codes, the padded code blocks and the units.  build_plan calls it after
// forming the groups; returns false with *err set on bad sizes.
bool plan_phase_solve(HostPlan *pl, std::string *err);

// S in storage order, 4 ints per entry (wx, wy, vx, vy).
void enumerate_S(int uc, int R, std::vector<int32_t> *wv);
// W in storage order, 2 ints per entry.
void enumerate_W(int uc, std::vector<int32_t> *w);
int count_shells(const std::vector<int32_t> &W);

}  // namespace nvsm
