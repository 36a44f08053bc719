// Internal layout shared by the host library and the gfx950 kernels.
//
// Work decomposition of the filter bank (§2.1, Eqs. 7-8):
//   * a workgroup owns L = 64*W lanes; each lane runs F filters of ONE
//     (template, band) segment, with the filter state in VGPRs;
//   * the segments of one band are laid end to end in lane space
//     (ceil(M/F) lanes each) and cut into workgroups of L lanes, so a segment
//     that straddles a workgroup boundary becomes two "pieces", each of which
//     writes its own partial band output to the workspace;
//   * per sample, each lane adds its F filters (pairwise), stores the partial
//     to LDS, and every kTile samples the workgroup reduces the partials of
//     each piece in two fixed-order levels (16-lane runs, then runs), so the
//     result does not depend on anything outside the bank.
#pragma once
#include <cstdint>

#include "spiir.h"

namespace spiir {

constexpr int kTile = 16;        // samples per reduction tile (R)
constexpr int kInnerBlock = 4096; // base-rate samples one launch sequence covers
constexpr int kRunLanes = 16;    // lanes per level-1 run group
constexpr int kMaxReq = SPIIR_MAX_BATCH;
constexpr int kMaxBands = SPIIR_MAX_BANDS;
constexpr int kMaxPiecesPerGroup = 128;
constexpr int kSlotNone = 0xffff;
// Matrix-core engine: samples per chunk, filters per workgroup (one lane
// each in the chunk chain), samples per output tile (16 chunks).
constexpr int kMfmaT = 8;
constexpr int kMfmaSlots = 256;
constexpr int kMfmaTile = 128;
// Size of the static workspace of spiir_process_block_noalloc.
constexpr size_t kScratchBytes = (size_t)SPIIR_NOALLOC_MAX_WORKSPACE;

// Largest workgroup of the filter kernel for F filters per lane: with 8
// filters a lane needs more than 128 VGPRs, so at most 2 waves per SIMD.
constexpr int filter_max_threads(int F) { return F >= 8 ? 512 : 1024; }
// Waves per SIMD the compiler must leave room for (caps VGPRs at 512 / n):
// with 4 filters and the plain sum a lane fits in 96 VGPRs (spills only
// outside the sample loop), so 5 waves; the compensated sum needs more, so 4.
// With 6 filters, 4 (128 VGPRs; again no spills in the sample loop).
constexpr int filter_min_waves(int F, bool comp) { return F == 4 ? (comp ? 4 : 5) : F == 6 ? 4 : 1; }

struct alignas(8) c32 {
    float x, y;
};
struct c64 {
    double x, y;
};

// One workgroup of the filter kernel.
struct WgDesc {
    int32_t band;
    int32_t maxd;        // largest delay among its filters: LDS window reach
    int32_t npiece;
    int32_t nrun;
    int64_t slot_base;   // filter slot (f, lane) lives at slot_base + f*L + lane
    int32_t meta_base;   // L lane-meta words: (piece << 16) | run slot (or kSlotNone)
    int32_t piece_base;  // first PieceDesc
    int32_t scale;       // matrix-core engine: log2 of the fp16 scale of its b0 a1^j
    int32_t pad;
};

// A contiguous lane range of one (template, band) segment inside a workgroup.
struct PieceDesc {
    int64_t zoff;  // workspace offset (complex elements) of its partial band output
    int32_t run0;  // its level-2 runs are [run0, run1) (workgroup-local)
    int32_t run1;
    int32_t tmpl;
    int32_t pad;
};

// Per (template, band): its pieces' outputs, consecutive with stride max_block >> h.
struct SegDesc {
    int64_t zoff;
    int32_t npiece;
    int32_t pad;
};

// Device-resident constant description of a bank (one copy per bank).
struct BankDev {
    int32_t T, H, L, F, C, precision;
    int32_t td, tu, hu_len, max_block;
    int32_t xcap;                   // LDS capacity of one window copy, floats
    int32_t copies;                 // window copies in LDS (1 or 2)
    int32_t nrun_max;               // level-2 run slots per tile row
    int32_t npiece_max;
    int32_t pad0;
    int32_t S[kMaxBands];           // window sub-block length per band
    int32_t ring_mask[kMaxBands];   // ring size - 1 per band (power of two)
    int64_t ring_off[kMaxBands];    // band ring offset in `rings`
    int64_t zstride[kMaxBands];     // workspace row length per band (even)
    int32_t band_wg0[kMaxBands + 1];
    const WgDesc* wg;
    const PieceDesc* piece;
    const SegDesc* seg;             // [T*H]
    const int32_t* lane_meta;
    // Slots of odd lanes hold the swapped form (see one_step): conj(fl32(a1)),
    // (Im b0, Re b0), conj(carry), and their states are (Im y, Re y).
    const c32* a;                   // per slot: fl32(a1)
    const c32* b;                   // per slot: fl32(b0)
    const c32* dc;                  // per slot: a1^C - fl32(a1)^C (FP64 -> FP32)
    const int32_t* off;             // per slot: delay d (band samples)
    c32* y;                         // per slot: state y[k-1]
    c32* ys;                        // per slot: pending carry correction dC * (state at the chunk start)
    float* rings;                   // per-band input history rings
    const float* hd;
    const float* hu;
    c32* zw;                        // the bank's own workspace (null with a caller workspace)
    c32* uphist;                    // [T][H][hu_len] last acc samples per band
    int32_t* flags;                 // [T] sticky non-finite flags
    // [0]: absolute base-rate index of the first sample of the chunk being
    // filtered; [1]: samples staged so far.  The staging kernel advances them,
    // so a recorded launch sequence can be replayed block after block.
    int64_t* clock;
    // Parallel-in-time split (P > 1): band h's samples are cut at absolute
    // multiples of lc[h] (a multiple of C) into at most P + 1 chunks per block.
    int32_t P;
    int32_t lc[kMaxBands];
    int64_t n_slots;
    const c32* al;                  // per slot: a1^lc (FP64 -> FP32), same form as `a`
    c32* uend;                      // [P+1][n_slots] chunk end states from zero start
    c32* schain;                    // [P+1][n_slots] chained chunk start states
    c32* ys0;                       // [n_slots] pending carry correction entering the block
    // Matrix-core engine (engine == SPIIR_ENGINE_MFMA): `a` holds fl32(a1^8),
    // `dc` the chunk-chain carry correction a1^C - fl32(a1^8)^(C/8), and
    //   kc[8*slot + j] = b0 a1^j, pw[8*slot + t] = a1^(t+1), j, t < 8.
    int32_t engine;
    const c32* kc;
    const c32* pw;
};

struct ReqArg {
    const BankDev* bd;
    const float* x;
    c32* zw;             // workspace: per-piece band outputs of the current chunk
    c32* z;              // null: the output is not written
    int64_t ldz;
    spiir_peak* peaks;   // null: no trigger reduction
    int32_t n;
    int32_t H;
    int32_t c0;          // offset of this chunk in the caller's block
    float thr2;          // threshold^2 of the trigger count
    int32_t nchunk;      // time-chunk slots per workgroup (1, or P + 1)
};

// Everything one launch sequence needs, passed by value as kernel arguments.
struct LaunchArgs {
    int32_t nreq;
    int32_t nseg;                                  // (band, request) WG ranges
    ReqArg req[kMaxReq];
    int32_t cum[kMaxReq * kMaxBands + 1];          // prefix of WG counts
    int16_t seg_req[kMaxReq * kMaxBands];
    int16_t seg_band[kMaxReq * kMaxBands];
    int32_t tcum[kMaxReq + 1];                     // prefix of templates
};

// Kernel arguments are limited to 4 KiB.
static_assert(sizeof(LaunchArgs) <= 4096, "launch arguments exceed the kernel argument limit");

// Launchers (spiir_kernels.hip).  All return hipError_t as int.
int launch_stage(const LaunchArgs& a, int lds_bytes, void* stream);
int launch_filter(int F, int precision, const LaunchArgs& a, int nblocks, int L, int lds_bytes,
                  void* stream);
int launch_filter_mfma(const LaunchArgs& a, int nblocks, int lds_bytes, void* stream);
int launch_upadd(const LaunchArgs& a, int nblocks, int lds_bytes, void* stream);
int launch_prep(const c64* a, const c64* b, int64_t n, int C, c32* fa, c32* fb, c32* fdc,
                const int32_t* slot_lc, c32* fal, void* stream);
int launch_filter_local(int F, int precision, const LaunchArgs& a, int nblocks, int L, int lds_bytes,
                        void* stream);
int launch_chain(const LaunchArgs& a, int64_t nblocks, void* stream);
int launch_fill(void* p, int64_t bytes, void* stream);
int filter_max_lds();
int allow_filter_lds();
// Address of the static workspace on `device`, which must be current
// (hipGetSymbolAddress once per device, then the kept address).
int scratch_ptr(int device, void** out);

}  // namespace spiir
