// Host side of the SPIIR library: descriptor validation, the lane/workgroup
// planner, device memory, launch sequencing, state and status.  Exposes the C
// ABI declared in include/spiir.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "spiir.h"
#include "spiir_internal.h"

using namespace spiir;

namespace {

// Default launch shape of a bank that fills the device (make_plan_fixed
// takes 4 filters per lane in 4-wave groups for the others): 4 filters per
// lane, 8 waves per group, with either sum.  The compensated sum's FP64
// cross-lane additions cost about what the plain ones do, so it gains nothing
// from covering more filters per lane (config 3, ms per block: F = 4, W = 8
// 1.122; F = 6, W = 4 1.168; F = 6, W = 8 1.194; F = 8, W = 4 1.333).
constexpr int kDefaultF = 4;
constexpr int kDefaultW = 8;
constexpr int kDefaultWWide = 4;  // with 6 or 8 filters per lane
constexpr int kDefaultC = 32;
constexpr int kSubBlock = 1024;     // samples per LDS window restage (largest tried)
constexpr int kNoFit = 1;           // internal: this launch shape exceeds the LDS budget
constexpr int kXcapMax = 24576;     // LDS window, floats
constexpr int kMaxLds = 160 * 1024;
constexpr int kComputeUnits = 256;  // MI355X
constexpr uint32_t kStateMagic = 0x53504952u;  // "SPIR"
constexpr uint32_t kStateVersion = 3;  // 3: 128-byte header with the layout fingerprint
constexpr int64_t kStateHeaderBytes = 128;

int default_filters_per_lane(const spiir_bank_desc* d)
{
    return d->filters_per_lane ? d->filters_per_lane : kDefaultF;
}

int default_waves_per_group(int F) { return F >= 6 ? kDefaultWWide : kDefaultW; }

int64_t next_pow2(int64_t v)
{
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

struct Plan {
    int T = 0, H = 0, L = 0, F = 0, W = 0, C = 0, precision = 0;
    int td = 0, tu = 0, hu_len = 0, max_block = 0, mb_inner = 0;
    int P = 1;
    int lc[SPIIR_MAX_BANDS] = {};
    int xcap = 0, copies = 2;
    int nrun_max = 1, npiece_max = 1;
    int lds_filter = 0, lds_stage = 0, lds_up = 0;
    int64_t total_filters = 0, n_slots = 0, zw_elems = 0, ring_total = 0;
    int workspace = SPIIR_WORKSPACE_OWN;
    int engine = SPIIR_ENGINE_VALU;
    int32_t n_groups = 0, n_pieces = 0;  // kept after the layout arrays are released
    std::vector<int> maxd_band, S, ring_mask;
    std::vector<int64_t> ring_off;
    std::vector<int64_t> zstride;   // workspace row per piece, per band (even length)
    std::vector<int> band_wg0;
    std::vector<WgDesc> wg;
    std::vector<PieceDesc> piece;
    std::vector<SegDesc> seg;
    std::vector<int32_t> lane_meta;
    std::vector<int64_t> slot_src;  // desc filter index, -1 = padding
    std::vector<int32_t> slot_off;
    size_t footprint = 0;
    uint64_t layout = 0;  // layout_fingerprint, taken before the arrays are released
};

bool finite_all(const double* p, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

int validate(const spiir_bank_desc* d)
{
    if (!d) return SPIIR_EINVAL;
    if (d->n_templates < 1 || d->n_bands < 1 || d->n_bands > SPIIR_MAX_BANDS) return SPIIR_EINVAL;
    if (d->base_rate_hz <= 0 || !d->n_filters) return SPIIR_EINVAL;
    const int H = d->n_bands;
    if (d->max_block <= 0 || d->max_block > (1 << 26)) return SPIIR_EINVAL;
    if (d->max_block % (1 << (H - 1)) != 0) return SPIIR_EINVAL;
    if (d->precision != SPIIR_FP32 && d->precision != SPIIR_FP32_COMPENSATED) return SPIIR_EINVAL;
    const int C = d->carry_chunk ? d->carry_chunk : kDefaultC;
    if (C < 16 || C > 1024 || (C & (C - 1)) != 0) return SPIIR_EINVAL;
    const int F = default_filters_per_lane(d);
    if (F != 1 && F != 2 && F != 4 && F != 6 && F != 8) return SPIIR_EINVAL;
    const int W = d->waves_per_group ? d->waves_per_group : default_waves_per_group(F);
    if (W < 1 || 64 * W > filter_max_threads(F)) return SPIIR_EINVAL;
    if (d->device < 0) return SPIIR_EINVAL;
    if (d->time_chunks != SPIIR_TIME_CHUNKS_AUTO &&
        (d->time_chunks < 0 || d->time_chunks > 64 || (d->time_chunks & (d->time_chunks - 1)) != 0))
        return SPIIR_EINVAL;
    if (d->window_copies < 0 || d->window_copies > 2) return SPIIR_EINVAL;
    if (d->workspace != SPIIR_WORKSPACE_OWN && d->workspace != SPIIR_WORKSPACE_CALLER) return SPIIR_EINVAL;
    if (d->engine != SPIIR_ENGINE_VALU && d->engine != SPIIR_ENGINE_MFMA) return SPIIR_EINVAL;
    if (d->engine == SPIIR_ENGINE_MFMA &&
        (H != 1 || d->precision != SPIIR_FP32 || d->max_block % kMfmaTile != 0 || d->time_chunks > 1))
        return SPIIR_EINVAL;
    int64_t total = 0;
    for (int64_t s = 0; s < (int64_t)d->n_templates * H; ++s) {
        if (d->n_filters[s] < 0) return SPIIR_EINVAL;
        total += d->n_filters[s];
    }
    if (total > 0) {
        if (!d->a1 || !d->b0 || !d->delay) return SPIIR_EINVAL;
        if (!finite_all(d->a1, 2 * total) || !finite_all(d->b0, 2 * total)) return SPIIR_EINVAL;
        for (int64_t l = 0; l < total; ++l)
            if (d->delay[l] < 0 || d->delay[l] > SPIIR_MAX_DELAY) return SPIIR_EINVAL;
    }
    if (H > 1) {
        if (d->n_taps_down < 1 || d->n_taps_down > SPIIR_MAX_TAPS || !d->h_down) return SPIIR_EINVAL;
        if (d->n_taps_up < 1 || d->n_taps_up > SPIIR_MAX_TAPS || !d->h_up) return SPIIR_EINVAL;
        if (!finite_all(d->h_down, d->n_taps_down) || !finite_all(d->h_up, d->n_taps_up))
            return SPIIR_EINVAL;
    }
    return SPIIR_OK;
}

// Lays out the bank: segments of each band end to end in lane space, cut into
// workgroups of L lanes; a segment crossing a workgroup boundary becomes two
// pieces.  Padding lanes and slots carry zero coefficients (their outputs are
// exactly zero) and belong to the last piece of their workgroup.
int make_plan_shape(const spiir_bank_desc* d, Plan& p, int W, int sub, int copies)
{
    p = Plan();
    p.T = d->n_templates;
    p.H = d->n_bands;
    p.F = default_filters_per_lane(d);
    p.W = W;
    p.L = 64 * p.W;
    p.C = d->carry_chunk ? d->carry_chunk : kDefaultC;
    p.precision = d->precision;
    p.workspace = d->workspace;
    p.max_block = d->max_block;
    p.mb_inner = std::min(d->max_block, kInnerBlock);
    p.td = p.H > 1 ? d->n_taps_down : 1;
    p.tu = p.H > 1 ? d->n_taps_up : 1;
    p.hu_len = (p.tu + 1) / 2;
    p.P = d->time_chunks > 1 ? d->time_chunks : 1;
    // chunk length per band: a multiple of C covering the band's share of the
    // largest launch in P pieces, so a block meets at most P + 1 chunks
    for (int h = 0; h < p.H; ++h) {
        const int mbh = std::max(p.mb_inner >> h, 1);
        const int per = (mbh + p.P - 1) / p.P;
        p.lc[h] = std::max(p.C, (per + p.C - 1) / p.C * p.C);
    }
    const int T = p.T, H = p.H, L = p.L, F = p.F;

    std::vector<int64_t> moff((size_t)T * H);
    int64_t total = 0;
    for (int64_t s = 0; s < (int64_t)T * H; ++s) {
        moff[s] = total;
        total += d->n_filters[s];
    }
    p.total_filters = total;

    p.maxd_band.assign(H, 0);
    for (int t = 0; t < T; ++t)
        for (int h = 0; h < H; ++h)
            for (int l = 0; l < d->n_filters[t * H + h]; ++l)
                p.maxd_band[h] = std::max(p.maxd_band[h], (int)d->delay[moff[t * H + h] + l]);

    // LDS window: one copy, or two (x and x shifted by one sample), of up to
    // maxd + S + 64 samples each, S = min(block, sub); with two, a copy's size
    // is 32 mod 64 dwords so that the second copy starts 32 banks after the
    // first.
    int X = 0;
    for (int h = 0; h < H; ++h)
        X = std::max(X, p.maxd_band[h] + std::min(sub, p.mb_inner >> h) + 65);
    X = copies == 2 ? ((X + 63) & ~63) + 32 : ((X + 63) & ~63);
    if (X > kXcapMax) return kNoFit;
    p.xcap = X;
    p.copies = copies;
    p.S.assign(H, 0);
    p.zstride.assign(H, 0);
    for (int h = 0; h < H; ++h) p.zstride[h] = (int64_t)(((p.mb_inner >> h) + 1) & ~1);
    p.ring_mask.assign(H, 0);
    p.ring_off.assign(H, 0);
    for (int h = 0; h < H; ++h) {
        const int nh = p.mb_inner >> h;
        p.S[h] = std::min(sub, nh);
        const int64_t P = next_pow2((int64_t)nh + std::max(p.maxd_band[h], p.td) + 1);
        p.ring_mask[h] = (int)(P - 1);
        p.ring_off[h] = p.ring_total;
        p.ring_total += P;
    }

    p.seg.assign((size_t)T * H, SegDesc{0, 0, 0});
    p.band_wg0.assign(H + 1, 0);

    struct Open {
        int lanes = 0;
        std::vector<int> lane_piece;  // piece (global index) per used lane
    } cur;
    std::vector<int64_t> wslot_src;   // slots of the open workgroup, [F][L]
    std::vector<int32_t> wslot_d;

    auto open_wg = [&]() {
        cur.lanes = 0;
        cur.lane_piece.clear();
        wslot_src.assign((size_t)F * L, -1);
        wslot_d.assign((size_t)F * L, 0);
    };
    auto close_wg = [&](int h) {
        if (cur.lanes == 0) return;
        WgDesc w{};
        w.band = h;
        w.slot_base = p.n_slots;
        w.meta_base = (int32_t)p.lane_meta.size();
        const int first_piece = cur.lane_piece.front();
        const int last_piece = cur.lane_piece.back();
        w.piece_base = first_piece;
        w.npiece = last_piece - first_piece + 1;
        int maxd = 0;
        for (int i = 0; i < F * L; ++i)
            if (wslot_src[i] >= 0) maxd = std::max(maxd, wslot_d[i]);
        w.maxd = maxd;
        // lane -> local piece (padding lanes join the last piece); runs end at a
        // piece change or at the end of each 16-lane group
        std::vector<int> lp(L);
        for (int i = 0; i < L; ++i)
            lp[i] = (i < cur.lanes ? cur.lane_piece[i] : last_piece) - first_piece;
        int run = 0;
        std::vector<int> run0(w.npiece, -1), run1(w.npiece, -1);
        for (int i = 0; i < L; ++i) {
            const bool end = (i % kRunLanes == kRunLanes - 1) || (i == L - 1) || lp[i + 1] != lp[i];
            int slot = kSlotNone;
            if (end) {
                slot = run++;
                if (run0[lp[i]] < 0) run0[lp[i]] = slot;
                run1[lp[i]] = slot + 1;
            }
            p.lane_meta.push_back((lp[i] << 16) | slot);
        }
        w.nrun = run;
        for (int q = 0; q < w.npiece; ++q) {
            p.piece[first_piece + q].run0 = run0[q];
            p.piece[first_piece + q].run1 = run1[q];
        }
        p.nrun_max = std::max(p.nrun_max, run);
        p.npiece_max = std::max(p.npiece_max, w.npiece);
        for (int i = 0; i < F * L; ++i) {
            p.slot_src.push_back(wslot_src[i]);
            p.slot_off.push_back(wslot_src[i] >= 0 ? wslot_d[i] : 0);
        }
        p.n_slots += (int64_t)F * L;
        p.wg.push_back(w);
        open_wg();
    };

    // Bank-aware placement.  With two window copies a full tile reads, per
    // filter, the 8-byte pair at x[k - d] from the copy of d's parity; with
    // the window origin a multiple of 64 samples and the copies 32 banks
    // apart, that read occupies the bank pair (15*(d & 1) - (d >> 1)) mod 32
    // plus a term common to all lanes.  64-bit reads are served 32 lanes at a
    // time over 64 banks, so within one half-wave and slot the lanes conflict
    // exactly when their classes agree.  With one copy the tile reads the
    // words x[k - d] and x[k + 1 - d] as two 32-bit accesses, served 32 lanes
    // at a time over 32 banks: there the class is (-d) mod 32 (two-copy
    // classes c and c + 16 of one parity would share a bank).  The two layouts
    // therefore place a bank's filters differently, and their outputs differ by
    // the order of the sum.  A segment's filters go to the (slot, half-wave)
    // rows of its lanes class by class, the classes with most filters first,
    // each filter to the row that holds fewest of its class so far (counting
    // the other segments sharing the row), ties to the row with most room.  A
    // segment's classes are uneven, so some rows must hold a class twice; this
    // order spreads the frequent classes before the rows fill (per filter slot
    // in lane order, least-used class first, left about 10% more conflict
    // cycles).
    constexpr int kBanks = 32;
    auto bank_class = [copies](int dj) {
        return copies == 2 ? (15 * (dj & 1) - (dj >> 1)) & (kBanks - 1) : (-dj) & (kBanks - 1);
    };
    const int halves = L / 32;
    using Counts = std::vector<uint16_t>;  // [F][halves][kBanks]
    auto fresh_counts = [&]() { return Counts((size_t)F * halves * kBanks, 0); };
    Counts cur_counts = fresh_counts();

    open_wg();
    for (int h = 0; h < H; ++h) {
        p.band_wg0[h] = (int)p.wg.size();
        const int64_t zstride = p.zstride[h];
        for (int t = 0; t < T; ++t) {
            const int M = d->n_filters[t * H + h];
            if (M == 0) continue;
            // an even number of lanes: lane pairs never straddle a run boundary
            const int nl = (((M + F - 1) / F) + 1) & ~1;
            const int64_t base = moff[t * H + h];

            // where the segment's lanes will land (mirrors the placement below)
            std::vector<int> lane_wg(nl), lane_pos(nl);
            {
                int lanes = cur.lanes;
                int pieces = cur.lanes ? cur.lane_piece.back() - cur.lane_piece.front() + 1 : 0;
                int wgid = 0, placed = 0;
                while (placed < nl) {
                    if (lanes == L || pieces >= kMaxPiecesPerGroup) {
                        ++wgid;
                        lanes = 0;
                        pieces = 0;
                    }
                    const int take = std::min(nl - placed, L - lanes);
                    ++pieces;
                    for (int i = 0; i < take; ++i) {
                        lane_wg[placed + i] = wgid;
                        lane_pos[placed + i] = lanes + i;
                    }
                    lanes += take;
                    placed += take;
                }
            }
            std::vector<Counts> counts(1, cur_counts);
            for (int i = 0; i < nl; ++i)
                while ((int)counts.size() <= lane_wg[i]) counts.push_back(fresh_counts());

            std::vector<std::vector<int>> bucket(kBanks);
            for (int j = M - 1; j >= 0; --j) {
                const int dj = d->delay[base + j];
                bucket[bank_class(dj)].push_back(j);
            }
            std::vector<int> assign((size_t)nl * F, -1);
            {
                // cells: (slot, half-wave row) of the segment's positions, each
                // with its positions in lane order
                struct Cell {
                    uint16_t* row;
                    std::vector<int> pos;  // i * F + f
                    int used = 0;
                };
                std::vector<Cell> cells;
                std::vector<int> cell_of_key;
                auto key_of = [&](int i, int f) {
                    return ((lane_wg[i] * F + f) * halves) + lane_pos[i] / 32;
                };
                int max_key = 0;
                for (int i = 0; i < nl; ++i)
                    for (int f = 0; f < F; ++f) max_key = std::max(max_key, key_of(i, f));
                cell_of_key.assign((size_t)max_key + 1, -1);
                for (int f = 0; f < F; ++f)
                    for (int i = 0; i < nl; ++i) {
                        if (i * F + f >= M) continue;  // padding positions: the tail of the last lane
                        const int k = key_of(i, f);
                        if (cell_of_key[k] < 0) {
                            cell_of_key[k] = (int)cells.size();
                            Cell c;
                            c.row = counts[lane_wg[i]].data() + ((size_t)f * halves + lane_pos[i] / 32) * kBanks;
                            cells.push_back(std::move(c));
                        }
                        cells[cell_of_key[k]].pos.push_back(i * F + f);
                    }
                // classes with the most filters first; each filter to the cell
                // holding fewest of its class so far, then the one with most room
                std::vector<int> order(kBanks);
                for (int r = 0; r < kBanks; ++r) order[r] = r;
                std::stable_sort(order.begin(), order.end(),
                                 [&](int a, int b) { return bucket[a].size() > bucket[b].size(); });
                for (int r : order)
                    while (!bucket[r].empty()) {
                        int best = -1;
                        for (int c = 0; c < (int)cells.size(); ++c) {
                            const Cell& C = cells[c];
                            const int room = (int)C.pos.size() - C.used;
                            if (room == 0) continue;
                            if (best < 0) { best = c; continue; }
                            const Cell& B = cells[best];
                            const int broom = (int)B.pos.size() - B.used;
                            if (C.row[r] < B.row[r] || (C.row[r] == B.row[r] && room > broom)) best = c;
                        }
                        Cell& C = cells[best];
                        assign[(size_t)C.pos[C.used++]] = bucket[r].back();
                        bucket[r].pop_back();
                        C.row[r]++;
                    }
            }

            SegDesc& sg = p.seg[(size_t)t * H + h];
            sg.zoff = p.zw_elems;
            sg.npiece = 0;
            int placed = 0, wg_seen = 0;
            while (placed < nl) {
                const int cur_pieces =
                    cur.lanes ? cur.lane_piece.back() - cur.lane_piece.front() + 1 : 0;
                if (cur.lanes == L || cur_pieces >= kMaxPiecesPerGroup) {
                    close_wg(h);
                    ++wg_seen;
                }
                const int take = std::min(nl - placed, L - cur.lanes);
                PieceDesc pc{};
                pc.zoff = p.zw_elems;
                pc.tmpl = t;
                p.zw_elems += zstride;
                const int pid = (int)p.piece.size();
                p.piece.push_back(pc);
                sg.npiece++;
                for (int i = 0; i < take; ++i) {
                    const int lane = cur.lanes + i;
                    for (int f = 0; f < F; ++f) {
                        const int j = assign[(size_t)(placed + i) * F + f];
                        if (j < 0) continue;
                        const int64_t src = base + j;
                        wslot_src[(size_t)f * L + lane] = src;
                        wslot_d[(size_t)f * L + lane] = d->delay[src];
                    }
                    cur.lane_piece.push_back(pid);
                }
                cur.lanes += take;
                placed += take;
            }
            cur_counts = counts[wg_seen];
        }
        close_wg(h);
        cur_counts = fresh_counts();
    }
    p.band_wg0[H] = (int)p.wg.size();
    // the kernel adds lane pairs before the run reduction: runs must end on odd lanes
    for (size_t i = 0; i < p.lane_meta.size(); ++i)
        if ((p.lane_meta[i] & 0xffff) != kSlotNone && (i & 1) == 0) return SPIIR_EINVAL;

    // The run-sum rows of the filter kernel's level 2 are nrun_max entries
    // apart; an odd stride keeps the 16 sample rows a level-1 store or a
    // level-2 read touches at once on distinct LDS bank pairs (an even stride
    // such as 24 made each such 64-bit store take 30 LDS cycles instead of 4).
    p.nrun_max |= 1;
    p.lds_filter = p.copies * p.xcap * 4 + (L / 2) * (kTile + 1) * 8 + 2 * kTile * p.nrun_max * 8 + p.npiece_max * 8 +
                   L * 4 + p.npiece_max * 8;
    p.lds_stage = ((p.td - 1) + p.mb_inner + (p.td - 1) + p.mb_inner / 2 + p.td) * 4;
    p.lds_up = (2 * (p.hu_len + p.mb_inner / 2) + std::max(p.H - 2, 0) * p.hu_len) * 8 + p.tu * 4;
    if (p.lds_stage > kMaxLds || p.lds_up > kMaxLds) return SPIIR_EINVAL;
    if (p.lds_filter > kMaxLds) return kNoFit;

    size_t fp = 0;
    fp += (size_t)p.n_slots * (5 * sizeof(c32) + sizeof(int32_t));
    fp += p.wg.size() * sizeof(WgDesc) + p.piece.size() * sizeof(PieceDesc);
    fp += p.seg.size() * sizeof(SegDesc) + p.lane_meta.size() * sizeof(int32_t);
    fp += (size_t)p.ring_total * sizeof(float) + (size_t)(p.td + p.tu) * sizeof(float);
    if (p.workspace == SPIIR_WORKSPACE_OWN) fp += (size_t)p.zw_elems * sizeof(c32);
    fp += (size_t)T * H * p.hu_len * sizeof(c32) + (size_t)T * sizeof(int32_t) + sizeof(BankDev);
    fp += 2 * sizeof(int64_t);
    if (p.P > 1)  // a1^lc, end states, chained states, entering chunk-start state, exponents
        fp += (size_t)p.n_slots * sizeof(c32) * (1 + 2 * (size_t)(p.P + 1) + 1);
    p.footprint = fp;
    p.n_groups = (int32_t)p.wg.size();
    p.n_pieces = (int32_t)p.piece.size();
    return SPIIR_OK;
}

// Waves per SIMD the registers of the filter kernel allow (from the compiled
// kernels' VGPR counts: 512 per SIMD lane over the rounded allocation); used
// only to rank launch shapes.
int filter_reg_waves(int F, bool comp)
{
    switch (F) {
    case 1: return comp ? 7 : 8;
    case 2: return 6;
    case 4: return comp ? 4 : 5;
    case 6: return 4;
    default: return 2;
    }
}

// Filter workgroups a compute unit runs at once for this bank: what the LDS
// and the registers allow, and no more than the bank's workgroups spread
// over the device's compute units.
int filter_groups_per_cu(const Plan& p)
{
    const int by_lds = kMaxLds / std::max(p.lds_filter, 1);
    const int by_regs = 4 * filter_reg_waves(p.F, p.precision == SPIIR_FP32_COMPENSATED) / p.W;
    const int64_t groups = (int64_t)p.wg.size() * p.P;
    const int by_bank = (int)std::min<int64_t>((groups + kComputeUnits - 1) / kComputeUnits, 1 << 20);
    return std::min(std::min(by_lds, by_regs), by_bank);
}

// Largest window sub-block for which the shape fits the LDS.
int fit_shape(const spiir_bank_desc* d, Plan& p, int W, int copies)
{
    int rc = kNoFit;
    for (int sub : {kSubBlock, 512, 256, 128, 64}) {
        rc = make_plan_shape(d, p, W, sub, copies);
        if (rc != kNoFit) return rc;
    }
    return rc;
}

// The launch shape: the caller's waves per group, or by default the shape's
// waves per group (8, or 4 with 6 or more filters per lane) and fewer when a
// bank's delay window does not fit the LDS (long delays); the window
// sub-block shrinks first.  The input window is held twice unless the caller
// asks for one copy, or a single copy lets a compute unit run more of the
// bank's waves where two leave it fewer than 3 per SIMD (long delay windows
// in banks large enough to fill the device); a copy less costs about 4% in
// LDS reads, more waves per SIMD gain more.
int make_plan_shaped(const spiir_bank_desc* d, Plan& p, int w_cap)
{
    int rc = validate(d);
    if (rc) return rc;
    const int F = default_filters_per_lane(d);
    std::vector<int> ws;
    if (d->waves_per_group)
        ws.push_back(d->waves_per_group);
    else
        for (int w : {8, 4, 2, 1})
            if (w <= w_cap && 64 * w <= filter_max_threads(F)) ws.push_back(w);
    for (int w : ws) {
        if (d->window_copies) {
            rc = fit_shape(d, p, w, d->window_copies);
            if (rc != kNoFit) return rc;
            continue;
        }
        rc = fit_shape(d, p, w, 2);
        if (rc != kNoFit && rc != SPIIR_OK) return rc;
        const int waves2 = rc == SPIIR_OK ? filter_groups_per_cu(p) * w : 0;
        if (waves2 >= 12) return SPIIR_OK;  // the one-copy plan is not needed
        Plan one;
        const int rc1 = fit_shape(d, one, w, 1);
        if (rc1 == kNoFit) {
            if (rc == kNoFit) continue;
            return SPIIR_OK;
        }
        if (rc1 != SPIIR_OK) return rc1;
        if (filter_groups_per_cu(one) * w > waves2) p = std::move(one);
        return SPIIR_OK;
    }
    return SPIIR_EINVAL;
}

// Rounds of workgroups the device runs for this plan: workgroups over
// workgroup slots (what the LDS and registers allow per compute unit, times
// the compute units).
double group_rounds(const Plan& p)
{
    const int by_lds = kMaxLds / std::max(p.lds_filter, 1);
    const int by_regs = 4 * filter_reg_waves(p.F, p.precision == SPIIR_FP32_COMPENSATED) / p.W;
    return (double)p.wg.size() / ((double)kComputeUnits * std::max(1, std::min(by_lds, by_regs)));
}

// The default launch shape (no filters_per_lane and no waves_per_group given).
// The shape that runs a full bank fastest (F = 4, W = 8) has large
// workgroups.  A bank that does not fill the device with them, or a
// multi-rate bank with fewer than 4 rounds of them (its band-0 workgroups, the
// longest, then decide when the block ends), runs faster in workgroups of 4
// waves: more, smaller workgroups balance better.  Measured, ms per block
// (F = 4, W = 8 -> F = 4, W = 4), compensated: config-3 banks of 1024, 2048,
// 3072, 4096 templates (1.2, 2.4, 3.6, 4.8 rounds) 0.68 -> 0.58, 0.86 -> 0.76,
// 1.10 -> 1.00, 1.25 -> 1.32; the uneven bank of 8192 templates (2.0 rounds)
// 1.33 -> 1.23; the single-rate bank of 1024 x 512 filters (1.0 round) 0.333 ->
// 0.346.  Plain, before the compensated sum moved to FP64: config-3 banks
// 0.71 -> 0.61, 0.93 -> 0.79, 1.19 -> 1.05, 1.32 -> 1.38; the uneven bank 1.31
// -> 1.21; the single-rate bank 0.348 -> 0.355.
int make_plan_fixed(const spiir_bank_desc* d, Plan& p)
{
    if (!d) return SPIIR_EINVAL;
    const int F = default_filters_per_lane(d);
    int rc = make_plan_shaped(d, p, default_waves_per_group(F));
    if (rc || d->filters_per_lane || d->waves_per_group) return rc;
    int bands_used = 0;
    for (int h = 0; h < p.H; ++h) bands_used += p.band_wg0[h + 1] > p.band_wg0[h];
    const double rounds = group_rounds(p);
    const double keep = bands_used > 1 ? 4.0 : 1.0;
    if (rounds >= keep || (p.F == 4 && p.W <= 4)) return SPIIR_OK;
    spiir_bank_desc d4 = *d;
    d4.filters_per_lane = 4;
    Plan small;
    if (make_plan_shaped(&d4, small, 4) != SPIIR_OK) return SPIIR_OK;
    p = std::move(small);
    return SPIIR_OK;
}

// Chunks for SPIIR_TIME_CHUNKS_AUTO.  A workgroup runs its band's samples of a
// block one after the other; the split cuts that sequence into about P pieces
// at the cost of an end-state pass.  It pays while the longest workgroup's
// sequence, cut in P, stays at least as long as the bank's work per workgroup
// slot of the device (work: the sum of every workgroup's band samples per
// block; slots: groups per compute unit times compute units).  Measured with
// the default shapes: single-rate banks of 64, 256 and 1024 templates of 512
// filters take P = 16, 4 and 1, the best of the powers of two tried; the
// multi-rate bank of 128, 512, 1024 and 4096 templates takes 16, 4, 2 and 1
// (also the best tried).
int auto_time_chunks(const Plan& p)
{
    int64_t work = 0;
    int64_t longest = 0;
    for (const WgDesc& w : p.wg) {
        const int64_t nh = std::max(p.mb_inner >> w.band, 1);
        work += nh;
        longest = std::max(longest, nh);
    }
    if (work == 0) return 1;
    const int by_lds = kMaxLds / std::max(p.lds_filter, 1);
    const int by_regs = 4 * filter_reg_waves(p.F, p.precision == SPIIR_FP32_COMPENSATED) / p.W;
    const int64_t slots = (int64_t)kComputeUnits * std::max(1, std::min(by_lds, by_regs));
    int P = 1;
    while (P < 64 && longest * slots >= 2 * P * work) P *= 2;
    return P;
}

// The matrix-core engine's layout (single-rate banks): every template's
// filters fill workgroups of kMfmaSlots slots, one template per workgroup
// (a template with more filters gets several, each a piece of its output),
// zero filters in the unused slots.  Each workgroup keeps the power-of-two
// scale that brings its largest |b0 a1^j| (j < 8) near 2^14 for its fp16
// coefficient operand.
int make_plan_mfma(const spiir_bank_desc* d, Plan& p)
{
    int rc = validate(d);
    if (rc) return rc;
    p = Plan();
    p.T = d->n_templates;
    p.H = 1;
    p.F = 1;
    p.W = kMfmaSlots / 64;
    p.L = kMfmaSlots;
    p.C = d->carry_chunk ? d->carry_chunk : kDefaultC;
    p.precision = d->precision;
    p.workspace = d->workspace;
    p.engine = SPIIR_ENGINE_MFMA;
    p.max_block = d->max_block;
    p.mb_inner = std::min(d->max_block, kInnerBlock);
    p.td = p.tu = 1;
    p.hu_len = 1;
    p.P = 1;
    p.lc[0] = p.C;
    p.copies = 2;
    const int T = p.T;
    int maxd = 0;
    int64_t total = 0;
    for (int t = 0; t < T; ++t) total += d->n_filters[t];
    p.total_filters = total;
    for (int64_t l = 0; l < total; ++l) maxd = std::max(maxd, (int)d->delay[l]);
    p.maxd_band.assign(1, maxd);
    // window sub-block: the longest of 512, 256, 128 samples whose window fits the LDS
    int sub = 0, X = 0;
    for (int sb : {512, 256, 128}) {
        sub = std::min(sb, p.mb_inner);
        // samples per window copy: 32 mod 128, so the copies' word offsets
        // are 16, 32 and 48 banks apart
        X = ((maxd + sub + 65 + 127) & ~127) + 32;
        if (4 * X * 2 + 2 * 16 * (kMfmaSlots + 4) * 4 + 4 * 16 * 17 * 4 <= kMaxLds) break;
    }
    if (X > kXcapMax) return SPIIR_EINVAL;
    p.xcap = X;
    p.S.assign(1, sub);
    p.zstride.assign(1, (int64_t)p.mb_inner);
    const int64_t ring = next_pow2((int64_t)p.mb_inner + std::max(maxd, 1) + 1);
    p.ring_mask.assign(1, (int)(ring - 1));
    p.ring_off.assign(1, 0);
    p.ring_total = ring;
    p.seg.assign((size_t)T, SegDesc{0, 0, 0});
    p.band_wg0.assign(2, 0);
    int64_t base = 0;
    for (int t = 0; t < T; ++t) {
        const int M = d->n_filters[t];
        SegDesc& sg = p.seg[t];
        sg.zoff = p.zw_elems;
        sg.npiece = 0;
        for (int f0 = 0; f0 < M; f0 += kMfmaSlots) {
            WgDesc w{};
            w.band = 0;
            w.npiece = 1;
            w.slot_base = p.n_slots;
            w.meta_base = (int32_t)p.lane_meta.size();
            w.piece_base = (int32_t)p.piece.size();
            int wmaxd = 0;
            double kmax = 0.0;
            // Bank-aware order: the chunk chain of slot i reads its 8 samples at
            // window position R - d from the copy of d's parity, whose 32-bit
            // word falls in bank (16 (d & 1) - (d + (d & 1)) / 2) mod 64 plus a
            // term common to all slots.  Each half-wave's 32 slots take filters
            // of the least-used bank so far in that half-wave.
            const int nf = std::min(kMfmaSlots, M - f0);
            std::vector<std::vector<int>> bucket(64);
            for (int f = nf - 1; f >= 0; --f) {
                const int dd = d->delay[base + f0 + f];
                bucket[((16 * (dd & 1) - (dd + (dd & 1)) / 2) % 64 + 64) % 64].push_back(f0 + f);
            }
            std::vector<int> order((size_t)kMfmaSlots, -1);
            for (int hw = 0; hw < kMfmaSlots / 32; ++hw) {
                int used[64] = {0};
                for (int i = 0; i < 32; ++i) {
                    int best = -1;
                    for (int c = 0; c < 64; ++c)
                        if (!bucket[c].empty() && (best < 0 || used[c] < used[best])) best = c;
                    if (best < 0) break;
                    order[hw * 32 + i] = bucket[best].back();
                    bucket[best].pop_back();
                    used[best]++;
                }
            }
            for (int i = 0; i < kMfmaSlots; ++i) {
                const int f = order[i];
                if (f >= 0) {
                    const int64_t src = base + f;
                    p.slot_src.push_back(src);
                    p.slot_off.push_back(d->delay[src]);
                    wmaxd = std::max(wmaxd, (int)d->delay[src]);
                    const double ar = d->a1[2 * src], ai = d->a1[2 * src + 1];
                    const double am = std::sqrt(ar * ar + ai * ai);
                    const double bm = std::hypot(d->b0[2 * src], d->b0[2 * src + 1]);
                    kmax = std::max(kmax, bm * std::max(1.0, std::pow(am, kMfmaT - 1)));
                } else {
                    p.slot_src.push_back(-1);
                    p.slot_off.push_back(0);
                }
                p.lane_meta.push_back(0);
            }
            w.maxd = wmaxd;
            w.scale = kmax > 0.0 ? 14 - (int)std::ceil(std::log2(kmax)) : 0;
            w.scale = std::max(-100, std::min(100, w.scale));
            PieceDesc pc{};
            pc.zoff = p.zw_elems;
            pc.tmpl = t;
            p.piece.push_back(pc);
            p.wg.push_back(w);
            p.zw_elems += p.zstride[0];
            p.n_slots += kMfmaSlots;
            sg.npiece++;
        }
        base += M;
    }
    p.band_wg0[1] = (int)p.wg.size();
    p.lds_filter = 4 * p.xcap * 2 + 2 * 16 * (kMfmaSlots + 4) * 4 + 4 * 16 * 17 * 4;
    p.lds_stage = ((p.td - 1) + p.mb_inner + (p.td - 1) + p.mb_inner / 2 + p.td) * 4;
    p.lds_up = (2 * (p.hu_len + p.mb_inner / 2)) * 8 + p.tu * 4;
    if (p.lds_filter > kMaxLds) return SPIIR_EINVAL;
    size_t fp = 0;
    fp += (size_t)p.n_slots * (5 * sizeof(c32) + sizeof(int32_t) + 2 * kMfmaT * sizeof(c32));
    fp += p.wg.size() * sizeof(WgDesc) + p.piece.size() * sizeof(PieceDesc);
    fp += p.seg.size() * sizeof(SegDesc) + p.lane_meta.size() * sizeof(int32_t);
    fp += (size_t)p.ring_total * sizeof(float) + (size_t)(p.td + p.tu) * sizeof(float);
    if (p.workspace == SPIIR_WORKSPACE_OWN) fp += (size_t)p.zw_elems * sizeof(c32);
    fp += (size_t)T * p.hu_len * sizeof(c32) + (size_t)T * sizeof(int32_t) + sizeof(BankDev);
    fp += 2 * sizeof(int64_t);
    p.footprint = fp;
    p.n_groups = (int32_t)p.wg.size();
    p.n_pieces = (int32_t)p.piece.size();
    return SPIIR_OK;
}

// The plan for a descriptor; an automatic time split plans the default (or
// given) shape first, then the same shape split in time.
int make_plan(const spiir_bank_desc* d, Plan& p)
{
    if (d && d->engine == SPIIR_ENGINE_MFMA) return make_plan_mfma(d, p);
    if (!d || d->time_chunks != SPIIR_TIME_CHUNKS_AUTO) return make_plan_fixed(d, p);
    spiir_bank_desc d1 = *d;
    d1.time_chunks = 0;
    int rc = make_plan_fixed(&d1, p);
    if (rc) return rc;
    const int P = auto_time_chunks(p);
    if (P < 2) return SPIIR_OK;
    d1.time_chunks = P;
    d1.filters_per_lane = p.F;
    d1.waves_per_group = p.W;
    d1.window_copies = p.copies;
    return make_plan_fixed(&d1, p);
}

// ---------------------------------------------------------------- profiling

struct ProfRec {
    int kind;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_recs;
std::vector<hipEvent_t> g_prof_pool;
spiir_profile_data g_prof_acc{};

hipEvent_t prof_event()
{
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Returns every event of the recorded launches to the pool once (consecutive
// launches share their boundary events).
void recycle_prof_events()
{
    std::vector<hipEvent_t> seen;
    for (auto& r : g_prof_recs) {
        if (std::find(seen.begin(), seen.end(), r.a) == seen.end()) seen.push_back(r.a);
        if (std::find(seen.begin(), seen.end(), r.b) == seen.end()) seen.push_back(r.b);
    }
    for (auto ev : seen) g_prof_pool.push_back(ev);
    g_prof_recs.clear();
}

}  // namespace

// ---------------------------------------------------------------- the bank

struct spiir_bank {
    Plan plan;
    int device = 0;
    int64_t done = 0;
    bool poisoned = false;
    hipEvent_t ev = nullptr;
    bool ev_recorded = false;
    // device memory
    c32 *a = nullptr, *b = nullptr, *dc = nullptr, *y = nullptr, *ys = nullptr;
    int32_t* off = nullptr;
    WgDesc* wg = nullptr;
    PieceDesc* piece = nullptr;
    SegDesc* seg = nullptr;
    int32_t* lane_meta = nullptr;
    float* rings = nullptr;
    float* hd = nullptr;
    float* hu = nullptr;
    c32* zw = nullptr;
    c32* uphist = nullptr;
    int32_t* flags = nullptr;
    int64_t* clock = nullptr;
    c32 *al = nullptr, *uend = nullptr, *schain = nullptr, *ys0 = nullptr;
    c32 *kc = nullptr, *pw = nullptr;  // matrix-core engine tables
    BankDev* bd = nullptr;
};

namespace {

template <class T>
hipError_t dalloc(T** p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void**)p, count * sizeof(T));
}

void free_bank(spiir_bank* b)
{
    if (!b) return;
    void* ptrs[] = {b->a,     b->b,     b->dc, b->y,  b->ys, b->off, b->wg,     b->piece, b->seg,
                    b->lane_meta, b->rings, b->hd, b->hu, b->zw, b->uphist, b->flags, b->clock, b->al, b->uend, b->schain, b->ys0,
                    b->kc, b->pw, b->bd};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    if (b->ev) (void)hipEventDestroy(b->ev);
    delete b;
}

int zero_state(spiir_bank* b, hipStream_t s)
{
    const Plan& p = b->plan;
    int e = 0;
    e |= launch_fill(b->y, p.n_slots * (int64_t)sizeof(c32), s);
    e |= launch_fill(b->ys, p.n_slots * (int64_t)sizeof(c32), s);
    e |= launch_fill(b->rings, p.ring_total * (int64_t)sizeof(float), s);
    e |= launch_fill(b->uphist, (int64_t)p.T * p.H * p.hu_len * (int64_t)sizeof(c32), s);
    e |= launch_fill(b->flags, (int64_t)p.T * (int64_t)sizeof(int32_t), s);
    e |= launch_fill(b->clock, 2 * (int64_t)sizeof(int64_t), s);
    return e;
}

// Bytes of one request's workspace (the per-piece band outputs of one chunk).
size_t workspace_bytes(const Plan& p)
{
    return ((size_t)p.zw_elems * sizeof(c32) + 255) & ~(size_t)255;
}

int64_t state_bytes(const Plan& p)
{
    return kStateHeaderBytes + p.n_slots * 2 * (int64_t)sizeof(c32) + p.ring_total * (int64_t)sizeof(float) +
           (int64_t)p.T * p.H * p.hu_len * (int64_t)sizeof(c32) + (int64_t)p.T * 4;
}

struct StateHeader {
    uint32_t magic, version;
    int32_t T, H, F, L, C, precision;
    int64_t n_slots, ring_total, done;
    int64_t hist;
    uint64_t layout;  // layout_fingerprint of the bank that wrote the blob
};
static_assert(sizeof(StateHeader) <= kStateHeaderBytes, "state header");

// FNV-1a over what decides where each value of the state lives: the filter
// behind every slot (its descriptor index and delay), the workgroup bands and
// the input ring sizes.  Banks of equal sizes whose delays place their filters
// differently get different fingerprints, so a blob cannot be loaded into them.
uint64_t layout_fingerprint(const Plan& p)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void* data, size_t bytes) {
        const unsigned char* c = static_cast<const unsigned char*>(data);
        for (size_t i = 0; i < bytes; ++i) {
            h ^= c[i];
            h *= 1099511628211ull;
        }
    };
    mix(p.slot_src.data(), p.slot_src.size() * sizeof(int64_t));
    mix(p.slot_off.data(), p.slot_off.size() * sizeof(int32_t));
    mix(p.band_wg0.data(), p.band_wg0.size() * sizeof(int));
    mix(p.ring_mask.data(), p.ring_mask.size() * sizeof(int));
    mix(&p.hu_len, sizeof(p.hu_len));
    mix(&p.engine, sizeof(p.engine));
    return h;
}

// peaks: the per-request trigger outputs (null for plain calls); with them a
// request may leave z_dev null.  static_ws: the library supplies the
// workspace (the requests' ws_dev are not looked at).
int validate_batch(int32_t n_req, const spiir_request* req, spiir_peak* const* peaks = nullptr,
                   bool static_ws = false)
{
    if (n_req < 1 || n_req > SPIIR_MAX_BATCH || !req) return SPIIR_EINVAL;
    for (int r = 0; r < n_req; ++r) {
        const spiir_request& q = req[r];
        if (!q.bank) return SPIIR_EINVAL;
        if (q.bank->poisoned) return SPIIR_EDEVICE;
        const Plan& p = q.bank->plan;
        if (q.n <= 0 || q.n > p.max_block || q.n % (1 << (p.H - 1)) != 0) return SPIIR_EINVAL;
        if (p.engine == SPIIR_ENGINE_MFMA && q.n % kMfmaTile != 0) return SPIIR_EINVAL;
        if (!q.x_dev) return SPIIR_EINVAL;
        if (peaks && !peaks[r]) return SPIIR_EINVAL;
        if (q.z_dev ? q.ldz < q.n : !peaks) return SPIIR_EINVAL;
        if (q.bank->device != req[0].bank->device) return SPIIR_EINVAL;
        if (!static_ws && (q.ws_dev ? ((uintptr_t)q.ws_dev & 255u) != 0 : !q.bank->zw)) return SPIIR_EINVAL;
        for (int s = 0; s < r; ++s)
            if (req[s].bank == q.bank) return SPIIR_EORDER;
    }
    return SPIIR_OK;
}

// The stream waits for each bank's previous work (per-bank order across streams).
hipError_t wait_banks(int32_t n_req, const spiir_request* req, hipStream_t s)
{
    hipError_t e = hipSuccess;
    for (int r = 0; r < n_req; ++r)
        if (req[r].bank->ev_recorded && e == hipSuccess) e = hipStreamWaitEvent(s, req[r].bank->ev, 0);
    return e;
}

// Test hook for the failure path: with SPIIR_TEST_FAIL_ENQUEUE set in the
// environment when the library loads, every launch sequence fails before its
// first launch (as a rejected launch would), so tests can reach the poisoned-
// bank path without a device fault.
const bool g_fail_enqueue = std::getenv("SPIIR_TEST_FAIL_ENQUEUE") != nullptr;

// Kernels of one batch on `s`: per inner chunk of at most kInnerBlock base-rate
// samples, the staging kernel (which advances each bank's device clock), the
// filter kernel and the upsample-and-add kernel.  Reads no host-side sample
// count, so a recorded sequence can be replayed.
hipError_t enqueue_batch(int32_t n_req, const spiir_request* req, hipStream_t s, bool prof,
                         spiir_peak* const* peaks = nullptr, float thr2 = 0.0f)
{
    hipError_t e = g_fail_enqueue ? hipErrorLaunchFailure : hipSuccess;
    int64_t maxn = 0;
    for (int r = 0; r < n_req; ++r) maxn = std::max<int64_t>(maxn, req[r].n);
    for (int64_t c0 = 0; c0 < maxn && e == hipSuccess; c0 += kInnerBlock) {
        LaunchArgs A;
        std::memset(&A, 0, sizeof(A));
        int rmap[SPIIR_MAX_BATCH];
        int lds_s = 0, lds_u = 0, ntm = 0, maxH = 0;
        for (int r = 0; r < n_req; ++r) {
            const spiir_request& q = req[r];
            if (q.n <= c0) continue;
            spiir_bank* b = q.bank;
            const Plan& p = b->plan;
            const int k = A.nreq++;
            rmap[k] = r;
            ReqArg& ra = A.req[k];
            ra.bd = b->bd;
            ra.x = q.x_dev + c0;
            ra.zw = q.ws_dev ? static_cast<c32*>(q.ws_dev) : b->zw;
            ra.z = q.z_dev ? reinterpret_cast<c32*>(q.z_dev) + c0 : nullptr;
            ra.ldz = q.ldz;
            ra.peaks = peaks ? peaks[r] : nullptr;
            ra.n = (int32_t)std::min<int64_t>(kInnerBlock, q.n - c0);
            ra.H = p.H;
            ra.c0 = (int32_t)c0;
            ra.thr2 = thr2;
            ra.nchunk = p.P > 1 ? p.P + 1 : 1;
            lds_s = std::max(lds_s, p.lds_stage);
            lds_u = std::max(lds_u, p.lds_up);
            maxH = std::max(maxH, p.H);
        }
        // one filter launch per launch shape (filters per lane, lanes, precision)
        // among the requests, in order of first appearance
        struct Shape {
            int F, L, prec, engine;
        };
        Shape shape_buf[kMaxReq];
        int nshape = 0;
        auto shape_of = [&](int k) {
            const Plan& p = req[rmap[k]].bank->plan;
            return Shape{p.F, p.L, p.precision, p.engine};
        };
        auto same = [](const Shape& a, const Shape& b) {
            return a.F == b.F && a.L == b.L && a.prec == b.prec && a.engine == b.engine;
        };
        for (int k = 0; k < A.nreq; ++k) {
            bool seen = false;
            for (int i = 0; i < nshape; ++i) seen |= same(shape_buf[i], shape_of(k));
            if (!seen) shape_buf[nshape++] = shape_of(k);
        }
        const Shape* const shapes_end = shape_buf + nshape;
        // filter workgroups of one shape: band-major across requests (longest
        // bands first), chunk-major inside a (band, request) segment when split
        // in time
        auto segments = [&](LaunchArgs& X, bool split_only, const Shape& sh) {
            int total = 0;
            X.nseg = 0;
            X.cum[0] = 0;
            for (int h = 0; h < maxH; ++h)
                for (int k = 0; k < X.nreq; ++k) {
                    const Plan& p = req[rmap[k]].bank->plan;  // X keeps A's request order
                    if (h >= p.H || !same(shape_of(k), sh)) continue;
                    if (split_only && X.req[k].nchunk == 1) continue;
                    const int cnt = (p.band_wg0[h + 1] - p.band_wg0[h]) * X.req[k].nchunk;
                    if (cnt == 0) continue;
                    X.seg_req[X.nseg] = (int16_t)k;
                    X.seg_band[X.nseg] = (int16_t)h;
                    X.cum[X.nseg + 1] = X.cum[X.nseg] + cnt;
                    X.nseg++;
                    total += cnt;
                }
            return total;
        };
        // time split: end-state passes and one chain pass (A2) over the split requests
        LaunchArgs A2;
        int64_t nchain = 0;
        bool split = false;
        for (int k = 0; k < A.nreq; ++k) split |= A.req[k].nchunk > 1;
        if (split) {
            std::memset(&A2, 0, sizeof(A2));
            for (int k = 0; k < A.nreq; ++k) {
                if (A.req[k].nchunk == 1) continue;
                const Plan& p = req[rmap[k]].bank->plan;
                A2.req[A2.nreq] = A.req[k];
                A2.cum[A2.nreq + 1] = A2.cum[A2.nreq] + (int32_t)((p.n_slots + 255) / 256);
                A2.nreq++;
            }
            nchain = A2.cum[A2.nreq];
        }
        A.tcum[0] = 0;
        for (int k = 0; k < A.nreq; ++k) {
            A.tcum[k + 1] = A.tcum[k] + req[rmap[k]].bank->plan.T;
            ntm += req[rmap[k]].bank->plan.T;
        }

        // kernel timing: kind 0 staging, kind 1 the filter bank (with the
        // time-split passes), kind 2 upsample-and-add
        hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
        auto mark = [&](int i) {
            if (!prof) return;
            ev[i] = prof_event();
            if (ev[i]) (void)hipEventRecord(ev[i], s);
        };
        // the LDS a shape's filter launch needs: the largest of its requests
        auto shape_lds = [&](const Shape& sh, bool split_only) {
            int lds = 0;
            for (int k = 0; k < A.nreq; ++k)
                if (same(shape_of(k), sh) && (!split_only || A.req[k].nchunk > 1))
                    lds = std::max(lds, req[rmap[k]].bank->plan.lds_filter);
            return lds;
        };
        mark(0);
        e = (hipError_t)launch_stage(A, lds_s, s);
        mark(1);
        if (split)
            for (const Shape* sp = shape_buf; sp != shapes_end; ++sp) {
                const Shape& sh = *sp;
                LaunchArgs X = A;
                const int n1 = segments(X, true, sh);
                if (e == hipSuccess && n1 > 0)
                    e = (hipError_t)launch_filter_local(sh.F, sh.prec, X, n1, sh.L, shape_lds(sh, true), s);
            }
        if (e == hipSuccess && split && nchain > 0) e = (hipError_t)launch_chain(A2, nchain, s);
        for (const Shape* sp = shape_buf; sp != shapes_end; ++sp) {
            const Shape& sh = *sp;
            LaunchArgs X = A;
            const int n0 = segments(X, false, sh);
            if (e == hipSuccess && n0 > 0)
                e = (hipError_t)(sh.engine == SPIIR_ENGINE_MFMA
                                     ? launch_filter_mfma(X, n0, shape_lds(sh, false), s)
                                     : launch_filter(sh.F, sh.prec, X, n0, sh.L, shape_lds(sh, false), s));
        }
        mark(2);
        if (e == hipSuccess) e = (hipError_t)launch_upadd(A, ntm, lds_u, s);
        mark(3);
        if (prof)
            for (int i = 0; i < 3; ++i)
                if (ev[i] && ev[i + 1]) g_prof_recs.push_back(ProfRec{i, ev[i], ev[i + 1]});
    }
    return e;
}

// Host bookkeeping after a batch was enqueued (or replayed): sample counts and
// per-bank completion events; a failed enqueue poisons the banks.
int finish_batch(int32_t n_req, const spiir_request* req, hipStream_t s, hipError_t e)
{
    if (e == hipSuccess)
        for (int r = 0; r < n_req; ++r) req[r].bank->done += req[r].n;
    for (int r = 0; r < n_req && e == hipSuccess; ++r) {
        e = hipEventRecord(req[r].bank->ev, s);
        req[r].bank->ev_recorded = true;
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        for (int r = 0; r < n_req; ++r) req[r].bank->poisoned = true;
        return SPIIR_EDEVICE;
    }
    return SPIIR_OK;
}

}  // namespace

// ---------------------------------------------------------------- recorded batches

struct spiir_graph {
    int device = 0;
    std::vector<spiir_request> req;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev = nullptr;  // recorded after each replay; destroy waits on it, not on the banks
    bool ev_recorded = false;
};

extern "C" {

const char* spiir_strerror(int status)
{
    switch (status) {
    case SPIIR_OK: return "ok";
    case SPIIR_EINVAL: return "invalid argument";
    case SPIIR_ENOMEM: return "out of device memory";
    case SPIIR_EDEVICE: return "device error (bank poisoned)";
    case SPIIR_EORDER: return "request order violated";
    case SPIIR_ENONFINITE: return "non-finite state or output";
    default: return "unknown status";
    }
}

static void fill_plan_info(const Plan& p, spiir_plan_info* info)
{
    info->total_filters = p.total_filters;
    info->filter_slots = p.n_slots;
    info->n_groups = p.n_groups;
    info->n_pieces = p.n_pieces;
    info->lanes_per_group = p.L;
    info->filters_per_lane = p.F;
    info->lds_bytes = p.lds_filter;
    info->carry_chunk = p.C;
    info->footprint = p.footprint;
    info->time_chunks = p.P;
    info->window_copies = p.copies;
    info->workspace_bytes = workspace_bytes(p);
    info->workspace = p.workspace;
    info->engine = p.engine;
}

int spiir_plan(const spiir_bank_desc* desc, spiir_plan_info* info)
{
    if (!info) return SPIIR_EINVAL;
    Plan p;
    int rc;
    try {
        rc = make_plan(desc, p);
    } catch (const std::bad_alloc&) {
        return SPIIR_ENOMEM;
    }
    if (rc) return rc;
    fill_plan_info(p, info);
    return SPIIR_OK;
}

int spiir_bank_plan(const spiir_bank* bank, spiir_plan_info* info)
{
    if (!bank || !info) return SPIIR_EINVAL;
    fill_plan_info(bank->plan, info);
    return SPIIR_OK;
}

int spiir_footprint(const spiir_bank_desc* desc, size_t* bytes)
{
    if (!bytes) return SPIIR_EINVAL;
    spiir_plan_info info;
    int rc = spiir_plan(desc, &info);
    if (rc) return rc;
    *bytes = info.footprint;
    return SPIIR_OK;
}

static c64 cmul_h(c64 u, c64 v) { return c64{u.x * v.x - u.y * v.y, u.x * v.y + u.y * v.x}; }

// Device arrays of a bank, sized from its plan (which may already have
// released its layout arrays: only counts are read here).
static bool alloc_bank(spiir_bank* b)
{
    const Plan& p = b->plan;
    bool ok = true;
    ok &= dalloc(&b->a, p.n_slots) == hipSuccess;
    ok &= dalloc(&b->b, p.n_slots) == hipSuccess;
    ok &= dalloc(&b->dc, p.n_slots) == hipSuccess;
    ok &= dalloc(&b->y, p.n_slots) == hipSuccess;
    ok &= dalloc(&b->ys, p.n_slots) == hipSuccess;
    ok &= dalloc(&b->off, p.n_slots) == hipSuccess;
    ok &= dalloc(&b->wg, p.n_groups) == hipSuccess;
    ok &= dalloc(&b->piece, p.n_pieces) == hipSuccess;
    ok &= dalloc(&b->seg, (size_t)p.T * p.H) == hipSuccess;
    ok &= dalloc(&b->lane_meta, (size_t)p.n_groups * p.L) == hipSuccess;
    ok &= dalloc(&b->rings, p.ring_total) == hipSuccess;
    ok &= dalloc(&b->hd, p.td) == hipSuccess;
    ok &= dalloc(&b->hu, p.tu) == hipSuccess;
    if (p.workspace == SPIIR_WORKSPACE_OWN) ok &= dalloc(&b->zw, p.zw_elems) == hipSuccess;
    ok &= dalloc(&b->uphist, (size_t)p.T * p.H * p.hu_len) == hipSuccess;
    ok &= dalloc(&b->flags, p.T) == hipSuccess;
    ok &= dalloc(&b->clock, 2) == hipSuccess;
    if (p.P > 1) {
        ok &= dalloc(&b->al, p.n_slots) == hipSuccess;
        ok &= dalloc(&b->uend, (size_t)(p.P + 1) * p.n_slots) == hipSuccess;
        ok &= dalloc(&b->schain, (size_t)(p.P + 1) * p.n_slots) == hipSuccess;
        ok &= dalloc(&b->ys0, p.n_slots) == hipSuccess;
    }
    if (p.engine == SPIIR_ENGINE_MFMA) {
        ok &= dalloc(&b->kc, (size_t)p.n_slots * kMfmaT) == hipSuccess;
        ok &= dalloc(&b->pw, (size_t)p.n_slots * kMfmaT) == hipSuccess;
    }
    ok &= dalloc(&b->bd, 1) == hipSuccess;
    ok &= hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) == hipSuccess;
    if (!ok) (void)hipGetLastError();
    return ok;
}

// The device-side description of a bank: its plan's sizes and its arrays.
static BankDev bank_dev(const spiir_bank* b)
{
    const Plan& p = b->plan;
    BankDev bd{};
    bd.T = p.T;
    bd.H = p.H;
    bd.L = p.L;
    bd.F = p.F;
    bd.C = p.C;
    bd.precision = p.precision;
    bd.td = p.td;
    bd.tu = p.tu;
    bd.hu_len = p.hu_len;
    bd.max_block = p.mb_inner;
    bd.xcap = p.xcap;
    bd.copies = p.copies;
    bd.nrun_max = p.nrun_max;
    bd.npiece_max = p.npiece_max;
    for (int h = 0; h < p.H; ++h) {
        bd.S[h] = p.S[h];
        bd.ring_mask[h] = p.ring_mask[h];
        bd.ring_off[h] = p.ring_off[h];
        bd.zstride[h] = p.zstride[h];
    }
    for (int h = 0; h <= p.H; ++h) bd.band_wg0[h] = p.band_wg0[h];
    bd.wg = b->wg;
    bd.piece = b->piece;
    bd.seg = b->seg;
    bd.lane_meta = b->lane_meta;
    bd.a = b->a;
    bd.b = b->b;
    bd.dc = b->dc;
    bd.off = b->off;
    bd.y = b->y;
    bd.ys = b->ys;
    bd.rings = b->rings;
    bd.hd = b->hd;
    bd.hu = b->hu;
    bd.zw = b->zw;
    bd.uphist = b->uphist;
    bd.flags = b->flags;
    bd.clock = b->clock;
    bd.P = p.P;
    for (int h = 0; h < p.H; ++h) bd.lc[h] = p.lc[h];
    bd.n_slots = p.n_slots;
    bd.al = b->al;
    bd.uend = b->uend;
    bd.schain = b->schain;
    bd.ys0 = b->ys0;
    bd.engine = p.engine;
    bd.kc = b->kc;
    bd.pw = b->pw;
    return bd;
}

// After upload the per-slot layout arrays live on the device only: the host
// keeps their fingerprint (state blobs) and counts, not the arrays.
static void release_layout(Plan& p)
{
    p.layout = layout_fingerprint(p);
    std::vector<WgDesc>().swap(p.wg);
    std::vector<PieceDesc>().swap(p.piece);
    std::vector<SegDesc>().swap(p.seg);
    std::vector<int32_t>().swap(p.lane_meta);
    std::vector<int64_t>().swap(p.slot_src);
    std::vector<int32_t>().swap(p.slot_off);
}

int spiir_create(const spiir_bank_desc* desc, void* stream, spiir_bank** out)
{
    if (!out) return SPIIR_EINVAL;
    *out = nullptr;
    spiir_bank* b = nullptr;
    try {
        b = new spiir_bank();
        int rc = make_plan(desc, b->plan);
        if (rc) {
            delete b;
            return rc;
        }
    } catch (const std::bad_alloc&) {
        delete b;
        return SPIIR_ENOMEM;
    }
    Plan& p = b->plan;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || desc->device >= ndev) {
        (void)hipGetLastError();
        delete b;
        return ndev == 0 ? SPIIR_EDEVICE : SPIIR_EINVAL;
    }
    b->device = desc->device;
    if (hipSetDevice(b->device) != hipSuccess || allow_filter_lds() != 0) {
        (void)hipGetLastError();
        delete b;
        return SPIIR_EDEVICE;
    }
    hipStream_t s = (hipStream_t)stream;
    if (!alloc_bank(b)) {
        free_bank(b);
        return SPIIR_ENOMEM;
    }

    // tables in lane order; coefficients go through the FP64 prep kernel
    c64* da = nullptr;
    c64* db = nullptr;
    std::vector<c64> ha, hb;
    try {
        ha.resize((size_t)p.n_slots);
        hb.resize((size_t)p.n_slots);
    } catch (const std::bad_alloc&) {
        free_bank(b);
        return SPIIR_ENOMEM;
    }
    for (int64_t g = 0; g < p.n_slots; ++g) {
        const int64_t src = p.slot_src[g];
        if (src >= 0) {
            ha[g] = c64{desc->a1[2 * src], desc->a1[2 * src + 1]};
            hb[g] = c64{desc->b0[2 * src], desc->b0[2 * src + 1]};
        } else {
            ha[g] = c64{0.0, 0.0};
            hb[g] = c64{0.0, 0.0};
        }
    }
    std::vector<float> hd(p.td, 1.0f), hu(p.tu, 1.0f);
    if (p.H > 1) {
        for (int i = 0; i < p.td; ++i) hd[i] = (float)desc->h_down[i];
        for (int i = 0; i < p.tu; ++i) hu[i] = (float)desc->h_up[i];
    }
    const BankDev bd = bank_dev(b);

    hipError_t e = hipSuccess;
    auto up = [&](void* dst, const void* src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    };
    if (hipMalloc((void**)&da, sizeof(c64) * std::max<int64_t>(p.n_slots, 1)) != hipSuccess ||
        hipMalloc((void**)&db, sizeof(c64) * std::max<int64_t>(p.n_slots, 1)) != hipSuccess) {
        if (da) (void)hipFree(da);
        if (db) (void)hipFree(db);
        (void)hipGetLastError();
        free_bank(b);
        return SPIIR_ENOMEM;
    }
    // time split: per-slot exponent of a1^lc (the slot's band chunk length)
    int32_t* dlc = nullptr;
    std::vector<int32_t> hlc;
    if (p.P > 1) {
        hlc.resize((size_t)p.n_slots);
        const int64_t per_wg = (int64_t)p.F * p.L;
        for (size_t w = 0; w < p.wg.size(); ++w)
            for (int64_t i = 0; i < per_wg; ++i) hlc[w * per_wg + i] = p.lc[p.wg[w].band];
        if (hipMalloc((void**)&dlc, sizeof(int32_t) * std::max<int64_t>(p.n_slots, 1)) != hipSuccess) {
            (void)hipFree(da);
            (void)hipFree(db);
            (void)hipGetLastError();
            free_bank(b);
            return SPIIR_ENOMEM;
        }
        up(dlc, hlc.data(), sizeof(int32_t) * p.n_slots);
    }
    up(da, ha.data(), sizeof(c64) * p.n_slots);
    up(db, hb.data(), sizeof(c64) * p.n_slots);
    up(b->off, p.slot_off.data(), sizeof(int32_t) * p.n_slots);
    up(b->wg, p.wg.data(), sizeof(WgDesc) * p.wg.size());
    up(b->piece, p.piece.data(), sizeof(PieceDesc) * p.piece.size());
    up(b->seg, p.seg.data(), sizeof(SegDesc) * p.seg.size());
    up(b->lane_meta, p.lane_meta.data(), sizeof(int32_t) * p.lane_meta.size());
    up(b->hd, hd.data(), sizeof(float) * p.td);
    up(b->hu, hu.data(), sizeof(float) * p.tu);
    up(b->bd, &bd, sizeof(BankDev));
    // matrix-core engine: its tables are FP64 powers rounded once, on the host
    std::vector<c32> ma, mz, mdc, mkc, mpw;
    if (p.engine == SPIIR_ENGINE_MFMA) {
        try {
            ma.resize((size_t)p.n_slots);
            mz.assign((size_t)p.n_slots, c32{0.0f, 0.0f});
            mdc.resize((size_t)p.n_slots);
            mkc.resize((size_t)p.n_slots * kMfmaT);
            mpw.resize((size_t)p.n_slots * kMfmaT);
        } catch (const std::bad_alloc&) {
            e = hipErrorOutOfMemory;
        }
        for (int64_t g = 0; g < p.n_slots && e == hipSuccess; ++g) {
            const c64 a = ha[g], bb = hb[g];
            c64 pw{1.0, 0.0};
            for (int j = 0; j < kMfmaT; ++j) {
                const c64 k = cmul_h(bb, pw);
                mkc[g * kMfmaT + j] = c32{(float)k.x, (float)k.y};
                pw = cmul_h(pw, a);
                mpw[g * kMfmaT + j] = c32{(float)pw.x, (float)pw.y};
            }
            // pw = a^8: the chunk-to-chunk factor, and the correction of its FP32
            // rounding over C samples, a^C - fl32(a^8)^(C/8), both in FP64
            const c32 a8{(float)pw.x, (float)pw.y};
            c64 exact{1.0, 0.0}, rounded{1.0, 0.0};
            const c64 a8r{a8.x, a8.y};
            for (int c = 0; c < p.C / kMfmaT; ++c) {
                exact = cmul_h(exact, pw);
                rounded = cmul_h(rounded, a8r);
            }
            ma[g] = a8;
            mdc[g] = c32{(float)(exact.x - rounded.x), (float)(exact.y - rounded.y)};
        }
        up(b->a, ma.data(), sizeof(c32) * p.n_slots);
        up(b->b, mz.data(), sizeof(c32) * p.n_slots);
        up(b->dc, mdc.data(), sizeof(c32) * p.n_slots);
        up(b->kc, mkc.data(), sizeof(c32) * p.n_slots * kMfmaT);
        up(b->pw, mpw.data(), sizeof(c32) * p.n_slots * kMfmaT);
    } else if (e == hipSuccess) {
        e = (hipError_t)launch_prep(da, db, p.n_slots, p.C, b->a, b->b, b->dc, dlc, b->al, s);
    }
    if (e == hipSuccess) e = (hipError_t)zero_state(b, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(da);
    (void)hipFree(db);
    if (dlc) (void)hipFree(dlc);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_bank(b);
        return SPIIR_EDEVICE;
    }
    release_layout(p);
    *out = b;
    return SPIIR_OK;
}

int spiir_clone(const spiir_bank* src, void* stream, spiir_bank** out)
{
    if (!out) return SPIIR_EINVAL;
    *out = nullptr;
    if (!src) return SPIIR_EINVAL;
    if (src->poisoned) return SPIIR_EDEVICE;
    spiir_bank* b = nullptr;
    try {
        b = new spiir_bank();
        b->plan = src->plan;  // sizes and counts only: the layout arrays were released
    } catch (const std::bad_alloc&) {
        delete b;
        return SPIIR_ENOMEM;
    }
    b->device = src->device;
    if (hipSetDevice(b->device) != hipSuccess) {
        (void)hipGetLastError();
        delete b;
        return SPIIR_EDEVICE;
    }
    if (!alloc_bank(b)) {
        free_bank(b);
        return SPIIR_ENOMEM;
    }
    const Plan& p = b->plan;
    hipStream_t s = (hipStream_t)stream;
    const BankDev bd = bank_dev(b);
    hipError_t e = src->ev_recorded ? hipStreamWaitEvent(s, src->ev, 0) : hipSuccess;
    auto dd = [&](void* dst, const void* from, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, from, bytes, hipMemcpyDeviceToDevice, s);
    };
    dd(b->a, src->a, sizeof(c32) * p.n_slots);
    dd(b->b, src->b, sizeof(c32) * p.n_slots);
    dd(b->dc, src->dc, sizeof(c32) * p.n_slots);
    dd(b->off, src->off, sizeof(int32_t) * p.n_slots);
    dd(b->wg, src->wg, sizeof(WgDesc) * p.n_groups);
    dd(b->piece, src->piece, sizeof(PieceDesc) * p.n_pieces);
    dd(b->seg, src->seg, sizeof(SegDesc) * (size_t)p.T * p.H);
    dd(b->lane_meta, src->lane_meta, sizeof(int32_t) * (size_t)p.n_groups * p.L);
    dd(b->hd, src->hd, sizeof(float) * p.td);
    dd(b->hu, src->hu, sizeof(float) * p.tu);
    if (p.P > 1) dd(b->al, src->al, sizeof(c32) * p.n_slots);
    if (p.engine == SPIIR_ENGINE_MFMA) {
        dd(b->kc, src->kc, sizeof(c32) * p.n_slots * kMfmaT);
        dd(b->pw, src->pw, sizeof(c32) * p.n_slots * kMfmaT);
    }
    if (e == hipSuccess && (e = hipMemcpyAsync(b->bd, &bd, sizeof(BankDev), hipMemcpyHostToDevice, s)) == hipSuccess)
        e = (hipError_t)zero_state(b, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_bank(b);
        return SPIIR_EDEVICE;
    }
    *out = b;
    return SPIIR_OK;
}

int spiir_process_batch(int32_t n_req, const spiir_request* req, void* stream)
{
    int rc = validate_batch(n_req, req);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(req[0].bank->device) != hipSuccess) return SPIIR_EDEVICE;
    hipError_t e = wait_banks(n_req, req, s);
    if (e == hipSuccess) {
        std::unique_lock<std::mutex> lk(g_prof_mu);
        const bool prof = g_prof_on;
        if (!prof) lk.unlock();
        e = enqueue_batch(n_req, req, s, prof);
    }
    return finish_batch(n_req, req, s, e);
}

int spiir_process_block(spiir_bank* bank, const float* x_dev, int64_t n, spiir_c32* z_dev,
                        int64_t ldz, void* stream)
{
    spiir_request r{bank, x_dev, n, z_dev, ldz, nullptr};
    return spiir_process_batch(1, &r, stream);
}

int spiir_process_block_noalloc(spiir_bank* bank, const float* x_dev, int64_t n, spiir_c32* z_dev,
                                int64_t ldz, void* stream)
{
    spiir_request r{bank, x_dev, n, z_dev, ldz, nullptr};
    int rc = validate_batch(1, &r, nullptr, true);
    if (rc) return rc;
    if (workspace_bytes(bank->plan) > kScratchBytes) return SPIIR_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(bank->device) != hipSuccess) return SPIIR_EDEVICE;
    if (scratch_ptr(bank->device, &r.ws_dev) != 0 || !r.ws_dev) {
        (void)hipGetLastError();
        return SPIIR_EDEVICE;
    }
    hipError_t e = wait_banks(1, &r, s);
    if (e == hipSuccess) e = enqueue_batch(1, &r, s, false);  // no timing events: they are created on demand
    return finish_batch(1, &r, s, e);
}

int spiir_process_batch_peaks(int32_t n_req, const spiir_request* req, spiir_peak* const* peak_dev,
                              float threshold, void* stream)
{
    if (!peak_dev || !(threshold >= 0.0f) || !std::isfinite(threshold)) return SPIIR_EINVAL;
    int rc = validate_batch(n_req, req, peak_dev);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(req[0].bank->device) != hipSuccess) return SPIIR_EDEVICE;
    hipError_t e = wait_banks(n_req, req, s);
    if (e == hipSuccess) {
        std::unique_lock<std::mutex> lk(g_prof_mu);
        const bool prof = g_prof_on;
        if (!prof) lk.unlock();
        const float thr2 = threshold * threshold;
        e = enqueue_batch(n_req, req, s, prof, peak_dev, thr2);
    }
    return finish_batch(n_req, req, s, e);
}

int spiir_process_peaks(spiir_bank* bank, const float* x_dev, int64_t n, spiir_c32* z_dev,
                        int64_t ldz, spiir_peak* peak_dev, float threshold, void* stream)
{
    spiir_request r{bank, x_dev, n, z_dev, ldz, nullptr};
    spiir_peak* pk[1] = {peak_dev};
    return spiir_process_batch_peaks(1, &r, pk, threshold, stream);
}

static int bank_sync(spiir_bank* b)
{
    if (hipSetDevice(b->device) != hipSuccess) return SPIIR_EDEVICE;
    if (b->ev_recorded && hipEventSynchronize(b->ev) != hipSuccess) {
        b->poisoned = true;
        return SPIIR_EDEVICE;
    }
    return SPIIR_OK;
}

int spiir_reset(spiir_bank* b)
{
    if (!b) return SPIIR_EINVAL;
    if (b->poisoned) return SPIIR_EDEVICE;
    int rc = bank_sync(b);
    if (rc) return rc;
    hipError_t e = (hipError_t)zero_state(b, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        b->poisoned = true;
        return SPIIR_EDEVICE;
    }
    b->done = 0;
    return SPIIR_OK;
}

int spiir_state_size(const spiir_bank* b, size_t* bytes)
{
    if (!b || !bytes) return SPIIR_EINVAL;
    *bytes = (size_t)state_bytes(b->plan);
    return SPIIR_OK;
}

int spiir_save_state(spiir_bank* b, void* host_buf, void* stream)
{
    if (!b || !host_buf) return SPIIR_EINVAL;
    if (b->poisoned) return SPIIR_EDEVICE;
    const Plan& p = b->plan;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(b->device) != hipSuccess) return SPIIR_EDEVICE;
    hipError_t e = hipSuccess;
    if (b->ev_recorded) e = hipStreamWaitEvent(s, b->ev, 0);
    StateHeader hdr{kStateMagic, kStateVersion, p.T, p.H, p.F, p.L, p.C, p.precision,
                    p.n_slots, p.ring_total, b->done, (int64_t)p.T * p.H * p.hu_len,
                    p.layout};
    char* o = (char*)host_buf;
    std::memset(o, 0, kStateHeaderBytes);
    std::memcpy(o, &hdr, sizeof(hdr));
    o += kStateHeaderBytes;
    auto dn = [&](const void* src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(o, src, bytes, hipMemcpyDeviceToHost, s);
        o += bytes;
    };
    dn(b->y, sizeof(c32) * p.n_slots);
    dn(b->ys, sizeof(c32) * p.n_slots);
    dn(b->rings, sizeof(float) * p.ring_total);
    dn(b->uphist, sizeof(c32) * (size_t)p.T * p.H * p.hu_len);
    dn(b->flags, sizeof(int32_t) * p.T);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        b->poisoned = true;
        return SPIIR_EDEVICE;
    }
    return SPIIR_OK;
}

int spiir_load_state(spiir_bank* b, const void* host_buf, void* stream)
{
    if (!b || !host_buf) return SPIIR_EINVAL;
    if (b->poisoned) return SPIIR_EDEVICE;
    const Plan& p = b->plan;
    StateHeader hdr;
    std::memcpy(&hdr, host_buf, sizeof(hdr));
    if (hdr.magic != kStateMagic || hdr.version != kStateVersion || hdr.T != p.T || hdr.H != p.H ||
        hdr.F != p.F || hdr.L != p.L || hdr.C != p.C || hdr.n_slots != p.n_slots ||
        hdr.ring_total != p.ring_total || hdr.hist != (int64_t)p.T * p.H * p.hu_len || hdr.done < 0 ||
        hdr.done % (1 << (p.H - 1)) != 0 || hdr.layout != p.layout)
        return SPIIR_EINVAL;
    int rc = bank_sync(b);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const char* o = (const char*)host_buf + kStateHeaderBytes;
    hipError_t e = hipSuccess;
    auto upl = [&](void* dst, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, o, bytes, hipMemcpyHostToDevice, s);
        o += bytes;
    };
    upl(b->y, sizeof(c32) * p.n_slots);
    upl(b->ys, sizeof(c32) * p.n_slots);
    upl(b->rings, sizeof(float) * p.ring_total);
    upl(b->uphist, sizeof(c32) * (size_t)p.T * p.H * p.hu_len);
    upl(b->flags, sizeof(int32_t) * p.T);
    const int64_t clk[2] = {hdr.done, hdr.done};
    if (e == hipSuccess) e = hipMemcpyAsync(b->clock, clk, sizeof(clk), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        b->poisoned = true;
        return SPIIR_EDEVICE;
    }
    b->done = hdr.done;
    return SPIIR_OK;
}

int spiir_status(spiir_bank* b, int32_t* template_flags)
{
    if (!b) return SPIIR_EINVAL;
    if (b->poisoned) return SPIIR_EDEVICE;
    int rc = bank_sync(b);
    if (rc) return rc;
    std::vector<int32_t> f(b->plan.T);
    if (hipMemcpy(f.data(), b->flags, sizeof(int32_t) * f.size(), hipMemcpyDeviceToHost) !=
        hipSuccess) {
        b->poisoned = true;
        return SPIIR_EDEVICE;
    }
    bool any = false;
    for (size_t t = 0; t < f.size(); ++t) {
        any |= f[t] != 0;
        if (template_flags) template_flags[t] = f[t] != 0;
    }
    return any ? SPIIR_ENONFINITE : SPIIR_OK;
}

int spiir_destroy(spiir_bank* b)
{
    if (!b) return SPIIR_OK;
    (void)hipSetDevice(b->device);
    if (b->ev_recorded) (void)hipEventSynchronize(b->ev);
    free_bank(b);
    return SPIIR_OK;
}

int spiir_graph_create(int32_t n_req, const spiir_request* req, spiir_graph** out)
{
    if (!out) return SPIIR_EINVAL;
    *out = nullptr;
    int rc = validate_batch(n_req, req);
    if (rc) return rc;
    if (hipSetDevice(req[0].bank->device) != hipSuccess) return SPIIR_EDEVICE;
    spiir_graph* g = nullptr;
    try {
        g = new spiir_graph();
        g->req.assign(req, req + n_req);
    } catch (const std::bad_alloc&) {
        delete g;
        return SPIIR_ENOMEM;
    }
    g->device = req[0].bank->device;
    hipStream_t cs = nullptr;
    hipError_t e = hipEventCreateWithFlags(&g->ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) {
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const hipError_t ee = enqueue_batch(n_req, req, cs, false);
            e = hipStreamEndCapture(cs, &g->graph);
            if (ee != hipSuccess) e = ee;
        }
        (void)hipStreamDestroy(cs);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (g->graph) (void)hipGraphDestroy(g->graph);
        if (g->ev) (void)hipEventDestroy(g->ev);
        delete g;
        return e == hipErrorOutOfMemory ? SPIIR_ENOMEM : SPIIR_EDEVICE;
    }
    *out = g;
    return SPIIR_OK;
}

int spiir_graph_launch(spiir_graph* g, void* stream)
{
    if (!g) return SPIIR_EINVAL;
    const int32_t n_req = (int32_t)g->req.size();
    for (const spiir_request& q : g->req)
        if (q.bank->poisoned) return SPIIR_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(g->device) != hipSuccess) return SPIIR_EDEVICE;
    hipError_t e = wait_banks(n_req, g->req.data(), s);
    if (e == hipSuccess) e = hipGraphLaunch(g->exec, s);
    if (e == hipSuccess) {
        e = hipEventRecord(g->ev, s);
        g->ev_recorded = e == hipSuccess;
    }
    return finish_batch(n_req, g->req.data(), s, e);
}

int spiir_graph_destroy(spiir_graph* g)
{
    if (!g) return SPIIR_OK;
    (void)hipSetDevice(g->device);
    if (g->ev_recorded) (void)hipEventSynchronize(g->ev);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->ev) (void)hipEventDestroy(g->ev);
    delete g;
    return SPIIR_OK;
}


int spiir_samples_done(const spiir_bank* b, int64_t* samples)
{
    if (!b || !samples) return SPIIR_EINVAL;
    *samples = b->done;
    return SPIIR_OK;
}

int spiir_profile_enable(int enable)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    recycle_prof_events();
    std::memset(&g_prof_acc, 0, sizeof(g_prof_acc));
    g_prof_on = enable != 0;
    return SPIIR_OK;
}

int spiir_profile_read(spiir_profile_data* out)
{
    if (!out) return SPIIR_EINVAL;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    int rc = SPIIR_OK;
    for (auto& r : g_prof_recs) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
            rc = SPIIR_EDEVICE;
            continue;
        }
        g_prof_acc.launches[r.kind] += 1;
        g_prof_acc.ms[r.kind] += ms;
    }
    recycle_prof_events();
    *out = g_prof_acc;
    return rc;
}

}  // extern "C"
