// gfx950 kernels of the SPIIR library.
//
//   k_stage   append a block to the band-0 input ring and run the /2 FIR
//             cascade (§2.2, resampling of Eq. 9 as a causal FIR) once per
//             stream, writing every band's new samples to its ring;
//   k_filter  the filter bank: Eq. 7 per filter with the state in VGPRs,
//             Eq. 8 as a deterministic two-level LDS reduction per piece;
//   k_upadd   per template: sum a band's pieces, add the x2 upsampled lower
//             band (§2.2, Fig. "multi"), lowest band first, write z;
//   k_prep    FP64 precompute of the carry corrections a1^C - fl32(a1)^C;
//   k_fill    zero fill (used instead of memset so the sequence stays a plain
//             chain of kernels).
#include <hip/hip_runtime.h>

#include <climits>
#include <mutex>
#include <type_traits>

#include "spiir_internal.h"

namespace spiir {

__device__ __forceinline__ float acc_fma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double acc_fma(double a, double b, double c) { return fma(a, b, c); }

// Address-space views of device memory.  Pointers held in the bank
// descriptor are generic; through a generic pointer the compiler emits flat
// accesses, which count against the LDS wait counter too, so a wait for an
// LDS read would also wait for every outstanding flat store or load.  Memory
// that no thread writes during a kernel (the descriptor, coefficient tables,
// input rings, the clock) is read through the constant view, which also lets
// uniform reads become scalar loads; memory a kernel writes, or reads and
// writes, goes through the global view.
#if defined(__HIP_DEVICE_COMPILE__)
#define SPIIR_AS_GLOBAL __attribute__((address_space(1)))
#define SPIIR_AS_CONST __attribute__((address_space(4)))
#else  // the host pass over this file only parses the kernels
#define SPIIR_AS_GLOBAL
#define SPIIR_AS_CONST
#endif
template <class T>
__device__ __forceinline__ SPIIR_AS_GLOBAL T* gmem(T* p)
{
    return (SPIIR_AS_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ const SPIIR_AS_CONST T* cmem(const T* p)
{
    return (const SPIIR_AS_CONST T*)p;
}
typedef const SPIIR_AS_CONST BankDev CBankDev;

// ---------------------------------------------------------------------------
// Input staging and the downsample cascade (one workgroup per request).
constexpr int kStageThreads = 1024;
constexpr int kStageFastTaps = 32;  // decimator length with an unrolled path
// LDS: cur [td-1 + max_block] | nxt [td-1 + max_block/2] | taps [td]
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kStageThreads) k_stage(LaunchArgs args)
{
    extern __shared__ float sm[];
    __shared__ long long s_base;
    const ReqArg& q = args.req[blockIdx.x];
    CBankDev* bd = cmem(q.bd);
    SPIIR_AS_GLOBAL int64_t* clock = gmem(bd->clock);
    const SPIIR_AS_GLOBAL float* x = gmem(q.x);
    const int n = q.n;
    if (threadIdx.x == 0) s_base = clock[1];
    __syncthreads();
    const int64_t s0 = s_base;
    if (threadIdx.x == 0) {
        clock[0] = s0;      // read by the filter kernel that follows
        clock[1] = s0 + n;
    }
    const int H = bd->H;
    SPIIR_AS_GLOBAL float* rings = gmem(bd->rings);
    SPIIR_AS_GLOBAL float* ring0 = rings + bd->ring_off[0];
    const int64_t m0 = bd->ring_mask[0];
    if (H == 1) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) ring0[(s0 + i) & m0] = x[i];
        return;
    }

    const int td = bd->td;
    const int hl = td - 1;
    const SPIIR_AS_CONST float* tap = cmem(bd->hd);
    float* cur = sm;
    float* nxt = sm + hl + bd->max_block;
    float* hd = nxt + hl + bd->max_block / 2;
    for (int i = threadIdx.x; i < td; i += blockDim.x) hd[i] = cmem(bd->hd)[i];
    for (int i = threadIdx.x; i < hl; i += blockDim.x) cur[i] = ring0[(s0 - hl + i) & m0];
    // the block goes to the band-0 ring and to LDS (the ring slots of the
    // history read above are not among the ones written here)
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const float v = x[i];
        ring0[(s0 + i) & m0] = v;
        cur[hl + i] = v;
    }
    __syncthreads();

    for (int h = 1; h < H; ++h) {
        const int nh = n >> h;
        const int64_t s0h = s0 >> h;
        SPIIR_AS_GLOBAL float* ring = rings + bd->ring_off[h];
        const int64_t mk = bd->ring_mask[h];
        if (h < H - 1)
            for (int i = threadIdx.x; i < hl; i += blockDim.x) nxt[i] = ring[(s0h - hl + i) & mk];
        for (int m = threadIdx.x; m < nh; m += blockDim.x) {
            // x_h[m] = sum_j h_d[j] x_{h-1}[2m - j]; cur[hl + i] holds x_{h-1} at block offset i
            const float* src = cur + hl + 2 * m;
            float s = 0.0f;
            if (td == kStageFastTaps) {
                // the common 32-tap decimator: taps as scalar loads, the window read
                // first, then the multiply-adds in the same order as the loop below
                float w[kStageFastTaps];
#pragma unroll
                for (int j = 0; j < kStageFastTaps; ++j) w[j] = src[-j];
#pragma unroll
                for (int j = 0; j < kStageFastTaps; ++j) s = fmaf(tap[j], w[j], s);
            } else {
                for (int j = 0; j < td; ++j) s = fmaf(hd[j], src[-j], s);
            }
            nxt[hl + m] = s;
            ring[(s0h + m) & mk] = s;
        }
        __syncthreads();
        float* t = cur;
        cur = nxt;
        nxt = t;
    }
}

// ---------------------------------------------------------------------------
// The filter bank.
// LDS: E0 [xcap] | E1 [xcap] (two copies only) | pbuf [L/2][kTile+1] c32 | l2 2 x [kTile][nrun_max] c32 |
//      pzoff [npiece_max] i64 | lmeta [L] i32 | prun [npiece_max] int2
// ---------------------------------------------------------------------------
// value of the other lane of the pair (lane ^ 1), via DPP quad_perm [1,0,3,2]
__device__ __forceinline__ float pair_swap(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
}

template <int F>
__device__ __forceinline__ void lane_sum(float (&vr)[F], float (&vi)[F])
{
    // pairwise tree over the lane's filters; the result is left in element 0
#pragma unroll
    for (int s = 1; s < F; s *= 2)
#pragma unroll
        for (int i = 0; i + s < F; i += 2 * s) {
            vr[i] += vr[i + s];
            vi[i] += vi[i + s];
        }
}

// One sample of Eq. 7 for the lane's F filters, given their inputs xv[f]; the
// lane sum is combined with the other lane of the pair and stored, one
// component per lane (the even lane the real part, the odd lane the imaginary
// part) at pcol[2*j].
//
// Odd lanes hold their filters in swapped form, (Im y, Re y), with the tables
// transformed to match (a1 -> conj(a1), b0 -> (Im b0, Re b0), carry ->
// conj): the same arithmetic then advances the swapped state.  So every
// lane's first component sum is what it keeps (even: Re, odd: Im) and its
// second is what its partner needs, and the pair combine is one DPP add.
template <int F, bool SUM>
__device__ __forceinline__ void one_step(const float (&xv)[F], float* __restrict__ pcol, int j,
                                         const float (&ar)[F],
                                         const float (&ai)[F], const float (&br)[F],
                                         const float (&bi)[F], float (&yr)[F], float (&yi)[F])
{
    float tr[F], ti[F];
#pragma unroll
    for (int f = 0; f < F; ++f) {
        const float pr = br[f] * xv[f], pi = bi[f] * xv[f];
        const float nr = fmaf(ar[f], yr[f], fmaf(-ai[f], yi[f], pr));
        const float ni = fmaf(ar[f], yi[f], fmaf(ai[f], yr[f], pi));
        yr[f] = nr; yi[f] = ni;
        tr[f] = nr; ti[f] = ni;
    }
    if (!SUM) return;  // end-state pass of a time split: no output
    lane_sum<F>(tr, ti);
    // even lane: re_even + re_odd; odd lane: im_odd + im_even
    pcol[2 * j] = tr[0] + pair_swap(ti[0]);
}

// A full tile of kTile samples starting at an absolute multiple of kTile.
// x2[f] points at the 8-byte aligned pair (x[k - d], x[k + 1 - d]) of filter f
// in the window copy of its delay's parity, so one ds_read_b64 feeds two
// samples.  Each pair stays one ds_read_b64: the pair is a native vector (a
// struct would be split into two 32-bit loads), and the scheduling barrier
// after each step's loads keeps the compiler from fusing the reads of
// consecutive pairs into ds_read2_b64.  On gfx950 a wave's ds_read_b64 whose
// 32-lane halves touch distinct bank pairs takes 2 LDS cycles, while a
// ds_read2_b64 over the same addresses took 15 (measured with
// SQ_LDS_IDX_ACTIVE and SQ_LDS_BANK_CONFLICT), so the fused form made the
// window reads the largest LDS cost and undid the bank-aware placement.  The
// barrier still lets the next step's loads be issued during this step's
// arithmetic.  The restrict qualifiers tell the compiler that the
// partial-sum stores never alias the window.
typedef float f32x2_t __attribute__((ext_vector_type(2)));
template <int F, bool SUM>
__device__ __forceinline__ void tile_full(const f32x2_t* const (&xp)[F], float* __restrict__ pcol,
                                          const float (&ar)[F],
                                          const float (&ai)[F], const float (&br)[F],
                                          const float (&bi)[F], float (&yr)[F], float (&yi)[F])
{
    const f32x2_t* __restrict__ x2[F];
#pragma unroll
    for (int f = 0; f < F; ++f) x2[f] = xp[f];
#pragma unroll
    for (int jj = 0; jj < kTile / 2; ++jj) {
        float xa[F], xb[F];
#pragma unroll
        for (int f = 0; f < F; ++f) {
            const f32x2_t v = x2[f][jj];
            xa[f] = v.x;
            xb[f] = v.y;
        }
        __builtin_amdgcn_sched_barrier(0);
        one_step<F, SUM>(xa, pcol, 2 * jj, ar, ai, br, bi, yr, yi);
        one_step<F, SUM>(xb, pcol, 2 * jj + 1, ar, ai, br, bi, yr, yi);
    }
}

// A full tile from a single window copy: x1[f] points at x[k - d]; each
// sample is one 32-bit read (the compiler pairs them into two-word reads).
template <int F, bool SUM>
__device__ __forceinline__ void tile_full1(const float* const (&xp)[F], float* __restrict__ pcol,
                                           const float (&ar)[F], const float (&ai)[F],
                                           const float (&br)[F], const float (&bi)[F],
                                           float (&yr)[F], float (&yi)[F])
{
    const float* __restrict__ x1[F];
#pragma unroll
    for (int f = 0; f < F; ++f) x1[f] = xp[f];
#pragma unroll
    for (int j = 0; j < kTile; ++j) {
        float xv[F];
#pragma unroll
        for (int f = 0; f < F; ++f) xv[f] = x1[f][j];
        one_step<F, SUM>(xv, pcol, j, ar, ai, br, bi, yr, yi);
    }
}

// `cnt` samples from arbitrary starting points: x1[f] points at x[k - d] in the
// unshifted window copy.
template <int F, bool SUM>
__device__ __forceinline__ void tile_partial(const float* const (&xp)[F], int cnt,
                                             float* __restrict__ pcol, const float (&ar)[F], const float (&ai)[F],
                                             const float (&br)[F], const float (&bi)[F],
                                             float (&yr)[F], float (&yi)[F])
{
    for (int j = 0; j < cnt; ++j) {
        float xv[F];
#pragma unroll
        for (int f = 0; f < F; ++f) xv[f] = xp[f][j];
        one_step<F, SUM>(xv, pcol, j, ar, ai, br, bi, yr, yi);
    }
}

// Time chunk c of a band's block [s0h, s0h + nh) when the bank is split in
// time: chunk 0 runs from the block start to the first absolute multiple of
// lc, chunk c >= 1 covers [B + (c-1) lc, B + c lc) clipped to the block.
struct Chunk {
    int k0, k1;       // block-relative sample range (empty if k0 >= k1)
    bool first, last; // first / last non-empty chunk of the block
};

__device__ __forceinline__ Chunk chunk_range(int c, int nchunk, int64_t s0h, int nh, int lc)
{
    Chunk r;
    if (nchunk == 1) {
        r.k0 = 0;
        r.k1 = nh;
        r.first = r.last = true;
        return r;
    }
    const int64_t B = (s0h + lc - 1) / lc * lc;
    const int first_c = B == s0h ? 1 : 0;
    const int last_c = s0h + nh - 1 < B ? 0 : 1 + (int)((s0h + nh - 1 - B) / lc);
    int64_t cs = c == 0 ? s0h : B + (int64_t)(c - 1) * lc;
    int64_t ce = c == 0 ? B : cs + lc;
    if (cs < s0h) cs = s0h;
    if (ce > s0h + nh) ce = s0h + nh;
    r.k0 = (int)(cs - s0h);
    r.k1 = ce > cs ? (int)(ce - s0h) : r.k0;
    r.first = c == first_c;
    r.last = c == last_c;
    return r;
}

constexpr int kStageBatch = 4;  // window loads a thread keeps in flight

// LOCAL: the end-state pass of a time split (every chunk but the last runs
// from zero, or the first from the carried state, and stores its end state;
// no output).  Otherwise: the filter pass proper, each chunk starting from its
// chained state.
template <int F, bool COMP, bool LOCAL>
__global__ void __launch_bounds__(filter_max_threads(F), filter_min_waves(F, COMP)) k_filter(LaunchArgs args)
{
    // Accumulator of the cross-lane sums: FP32 for the plain sum, FP64 for the
    // compensated one.
    using Acc = typename std::conditional<COMP, double, float>::type;
    extern __shared__ float sm[];
    const int bid = blockIdx.x;
    int lo = 0, hi = args.nseg;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (args.cum[mid] <= bid) lo = mid;
        else hi = mid;
    }
    const ReqArg& q = args.req[args.seg_req[lo]];
    const int h = args.seg_band[lo];
    CBankDev* bd = cmem(q.bd);
    const int nwg_h = bd->band_wg0[h + 1] - bd->band_wg0[h];
    const int li = bid - args.cum[lo];
    const int tc = li / nwg_h;  // time chunk (chunk-major order)
    const WgDesc wg = cmem(bd->wg)[bd->band_wg0[h] + (li - tc * nwg_h)];
    const int L = blockDim.x;
    const int tid = threadIdx.x;
    const int nh = q.n >> h;
    const int64_t s0h = cmem(bd->clock)[0] >> h;  // set by the staging kernel of this chunk
    const Chunk ch = chunk_range(tc, q.nchunk, s0h, nh, bd->lc[h]);
    if (ch.k0 >= ch.k1 || (LOCAL && ch.last)) return;  // whole workgroup
    const int64_t cmask = bd->C - 1;
    const int nrun = bd->nrun_max;

    // The x window is held twice, E0[m] = x[origin + m] and E1[m] = x[origin + 1 + m]
    // (origin a multiple of 64 absolute samples, E1 32 banks after E0), or once (E0).
    const bool two_copies = bd->copies == 2;
    float* E0 = sm;
    float* E1 = sm + bd->xcap;
    c32* pbuf = reinterpret_cast<c32*>(sm + bd->copies * bd->xcap);
    c32* l2buf = pbuf + (L / 2) * (kTile + 1);  // two tile buffers of run sums
    long long* pzoff = reinterpret_cast<long long*>(l2buf + 2 * kTile * nrun);
    int* lmeta = reinterpret_cast<int*>(pzoff + bd->npiece_max);
    int2* prun = reinterpret_cast<int2*>(lmeta + L);

    lmeta[tid] = cmem(bd->lane_meta)[wg.meta_base + tid];
    for (int p = tid; p < wg.npiece; p += L) {
        const PieceDesc pd = cmem(bd->piece)[wg.piece_base + p];
        pzoff[p] = pd.zoff;
        prun[p] = make_int2(pd.run0, pd.run1);
    }

    float ar[F], ai[F], br[F], bi[F], dr[F], di[F], yr[F], yi[F], ur[F], ui[F];
    int dl[F];
    // Start state: y and the pending carry correction u = dC * (y at the start
    // of the current carry chunk), which is added to y at the chunk's end.
    // The first chunk starts from the carried state; when the block has more
    // than one chunk, the end-state pass saves that state (schain row of the
    // first chunk, ys0) for the filter pass, whose last chunk overwrites the
    // carried state while the first may still read it.  A later chunk starts
    // from zero in the end-state pass and from its chained state in the
    // filter pass; its start is a carry-chunk boundary, so u = dC * y there.
    const c32* ysrc = bd->y;
    const c32* yssrc = bd->ys;
    if (!ch.first) ysrc = yssrc = bd->schain + (int64_t)tc * bd->n_slots;
    else if (!LOCAL && !ch.last) {
        ysrc = bd->schain + (int64_t)tc * bd->n_slots;
        yssrc = bd->ys0;
    }
    const SPIIR_AS_GLOBAL c32* ysg = gmem(ysrc);
    const SPIIR_AS_GLOBAL c32* yssg = gmem(yssrc);
#pragma unroll
    for (int f = 0; f < F; ++f) {
        const int64_t g = wg.slot_base + (int64_t)f * L + tid;
        c32 y = ysg[g], ys = yssg[g];
        if (LOCAL && !ch.first) y = ys = c32{0.0f, 0.0f};
        if (LOCAL && ch.first) {
            gmem(bd->schain)[(int64_t)tc * bd->n_slots + g] = y;
            gmem(bd->ys0)[g] = ys;
        }
        const c32 a = cmem(bd->a)[g], b = cmem(bd->b)[g], d = cmem(bd->dc)[g];
        ar[f] = a.x; ai[f] = a.y;
        br[f] = b.x; bi[f] = b.y;
        dr[f] = d.x; di[f] = d.y;
        yr[f] = y.x; yi[f] = y.y;
        if (ch.first) {
            ur[f] = ys.x; ui[f] = ys.y;
        } else {
            ur[f] = fmaf(d.x, y.x, -d.y * y.y);
            ui[f] = fmaf(d.x, y.y, d.y * y.x);
        }
        dl[f] = cmem(bd->off)[g];
    }
    __syncthreads();

    // level-1 role: sample row j1 of the 16-lane group q1; runs end where endmask
    // is set.  A wave reduces its own four groups; the first half-wave takes
    // groups 0 and 2 of them and the second 1 and 3, so that the two groups one
    // 32-lane half reads are 16 pair entries apart, 32 banks apart in the
    // [L/2][kTile+1] tile, and its 64-bit reads never share a bank pair.
    const int j1 = tid & (kTile - 1);
    const int q1 = (tid >> 6) * 4 + (((tid >> 4) & 1) << 1) + ((tid >> 5) & 1);
    unsigned endmask = 0;
    int slot0 = -1;
#pragma unroll
    for (int i = 0; i < kRunLanes / 2; ++i) {
        const int sl = lmeta[q1 * kRunLanes + 2 * i + 1] & 0xffff;
        if (sl != kSlotNone) {
            endmask |= 1u << i;
            if (slot0 < 0) slot0 = sl;
        }
    }
    // The single-run form applies when every 16-lane group the wave reduces is
    // one run; otherwise the whole wave takes the segmented form (which also
    // handles single-run groups), so no wave executes both.
    const bool wave_single_run = __all(endmask == (1u << (kRunLanes / 2 - 1)));

    const int S = bd->S[h];
    const SPIIR_AS_CONST float* ring = cmem(bd->rings) + bd->ring_off[h];
    const int64_t mk = bd->ring_mask[h];
    SPIIR_AS_GLOBAL c32* zwg = gmem(q.zw);
    // Lanes come in pairs of one run (segments span an even number of lanes).
    // The pair sum of sample j is entry e = lane/2 of row j: pbuf[e*(kTile+1) + j],
    // the even lane storing its real part and the odd lane its imaginary part.
    const int pe = tid >> 1;
    float* pcol = reinterpret_cast<float*>(pbuf + pe * (kTile + 1)) + (tid & 1);
    int parity = 0;

    for (int kb = ch.k0; kb < ch.k1; kb += S) {
        const int sub = min(S, ch.k1 - kb);
        // window start: a multiple of 64 at or below the oldest sample any filter
        // reads, minus one, so that an odd-delay pair never starts before E1[0]
        const int64_t origin = ((s0h + kb - wg.maxd - 1) >> 6) << 6;
        const int wn = (int)(s0h + kb + sub - origin);
        __syncthreads();
        // kStageBatch loads in flight per thread before their LDS stores
        for (int i0 = tid; i0 <= wn; i0 += kStageBatch * L) {
            float v[kStageBatch];
#pragma unroll
            for (int u = 0; u < kStageBatch; ++u) {
                const int i = i0 + u * L;
                v[u] = i <= wn ? ring[(origin + i) & mk] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < kStageBatch; ++u) {
                const int i = i0 + u * L;
                if (i < wn) E0[i] = v[u];
                if (two_copies && i > 0 && i <= wn) E1[i - 1] = v[u];
            }
        }
        __syncthreads();

        int k = kb;
        while (k < kb + sub) {
            const int64_t kabs = s0h + k;
            int cnt = kTile - (int)(kabs & (kTile - 1));
            if (cnt > kb + sub - k) cnt = kb + sub - k;
            const int rel = (int)(kabs - origin);  // window position of sample k
            if (cnt == kTile && two_copies) {
                const f32x2_t* xp[F];
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    const int par = dl[f] & 1;
                    xp[f] = reinterpret_cast<const f32x2_t*>((par ? E1 : E0) + (rel - dl[f] - par));
                }
                tile_full<F, !LOCAL>(xp, pcol, ar, ai, br, bi, yr, yi);
            } else if (cnt == kTile) {
                const float* xp[F];
#pragma unroll
                for (int f = 0; f < F; ++f) xp[f] = E0 + (rel - dl[f]);
                tile_full1<F, !LOCAL>(xp, pcol, ar, ai, br, bi, yr, yi);
            } else {
                const float* xp[F];
#pragma unroll
                for (int f = 0; f < F; ++f) xp[f] = E0 + (rel - dl[f]);
                tile_partial<F, !LOCAL>(xp, cnt, pcol, ar, ai, br, bi, yr, yi);
            }

            // carry correction after the last sample of an absolute chunk of C
            // samples: add the pending correction, then form the next chunk's
            // from the corrected state (each value keeps its own registers)
            if (((kabs + cnt) & cmask) == 0) {
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    yr[f] += ur[f];
                    yi[f] += ui[f];
                    ur[f] = fmaf(dr[f], yr[f], -di[f] * yi[f]);
                    ui[f] = fmaf(dr[f], yi[f], di[f] * yr[f]);
                }
            }

            if (!LOCAL) {
                // Level 1 reads only partials written by the thread's own wave (its
                // 16-lane group lies inside the wave), so a wave-local sync suffices.
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                c32* l2 = l2buf + parity * (kTile * nrun);
                // level 1: each thread sums one sample row over the runs of a 16-lane group
                // (all 16 partials are loaded before any run result is stored); each run
                // sum is rounded to FP32 once
                if (j1 < cnt) {
                    constexpr int kPairs = kRunLanes / 2;
                    const int e0 = q1 * kPairs;
                    const c32* grp = pbuf + e0 * (kTile + 1) + j1;
                    // one ds_read_b64 each (the barriers keep the compiler from
                    // pairing them into ds_read2_b64, which takes twice as long)
                    c32 v[kPairs];
    #pragma unroll
                    for (int i = 0; i < kPairs; ++i) {
                        v[i] = grp[i * (kTile + 1)];
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    c32* out = l2 + j1 * nrun;
                    if (wave_single_run) {
                        // the whole group is one run: a pairwise tree (short dependency chains)
                        Acc tr[kPairs], ti[kPairs];
    #pragma unroll
                        for (int i = 0; i < kPairs; ++i) {
                            tr[i] = v[i].x;
                            ti[i] = v[i].y;
                        }
    #pragma unroll
                        for (int st = 1; st < kPairs; st *= 2)
    #pragma unroll
                            for (int i = 0; i + st < kPairs; i += 2 * st) {
                                tr[i] += tr[i + st];
                                ti[i] += ti[i + st];
                            }
                        out[slot0] = c32{(float)tr[0], (float)ti[0]};
                    } else {
                        // runs in order; the accumulator restarts after a run end by a
                        // multiplication with keep = 0 (exact, and no selects)
                        int slot = slot0;
                        Acc accr = v[0].x, acci = v[0].y;
    #pragma unroll
                        for (int i = 0; i < kPairs; ++i) {
                            if (i > 0) {
                                const Acc keep = (Acc)(((endmask >> (i - 1)) & 1u) ^ 1u);
                                accr = acc_fma(accr, keep, (Acc)v[i].x);
                                acci = acc_fma(acci, keep, (Acc)v[i].y);
                            }
                            if ((endmask >> i) & 1u) {
                                out[slot] = c32{(float)accr, (float)acci};
                                ++slot;
                            }
                        }
                    }
                }
                __syncthreads();
                // level 2: each (piece, sample) sums its runs in order and writes the output
                for (int task = tid; task < wg.npiece * kTile; task += L) {
                    const int p = task / kTile;
                    const int j = task & (kTile - 1);
                    if (j < cnt) {
                        const int2 rr = prun[p];
                        const c32* row = l2 + j * nrun;
                        Acc accr = 0, acci = 0;
                        for (int s = rr.x; s < rr.y; ++s) {
                            const c32 v = row[s];
                            accr += v.x;
                            acci += v.y;
                        }
                        zwg[pzoff[p] + k + j] = c32{(float)accr, (float)acci};
                    }
                }
            }
            parity ^= 1;
            k += cnt;
        }
    }

    if (LOCAL) {
        SPIIR_AS_GLOBAL c32* ue = gmem(bd->uend) + (int64_t)tc * bd->n_slots;
#pragma unroll
        for (int f = 0; f < F; ++f) ue[wg.slot_base + (int64_t)f * L + tid] = c32{yr[f], yi[f]};
        return;
    }
    if (!ch.last) return;  // only the block's last chunk carries its state on
    bool bad = false;
#pragma unroll
    for (int f = 0; f < F; ++f) {
        const int64_t g = wg.slot_base + (int64_t)f * L + tid;
        gmem(bd->y)[g] = c32{yr[f], yi[f]};
        gmem(bd->ys)[g] = c32{ur[f], ui[f]};
        bad |= !(isfinite(yr[f]) && isfinite(yi[f]));
    }
    if (bad) {
        const int p = lmeta[tid] >> 16;
        atomicOr(&bd->flags[cmem(bd->piece)[wg.piece_base + p].tmpl], 1);
    }
}

// ---------------------------------------------------------------------------
// The filter bank on the matrix cores (single-rate banks; engine MFMA).
//
// Over a chunk of T = 8 samples starting at an absolute multiple of 8 (c is
// the chunk, Y_l[c] filter l's state before it), Eq. 6 applied to Eq. 7 gives
//   y_l[8c + t] = a_l^(t+1) Y_l[c] + sum_{s<=t} b_l a_l^(t-s) x[8c + s - d_l],
// so the sum over filters (Eq. 8) of one chunk is two matrix products with
// rows (t, re/im): a 16 x (2 per filter) block of powers a_l^(t+1) times the
// chunk states, and a 16 x (8 per filter) lower-triangular Toeplitz block of
// b_l a_l^(t-s) times the chunk's delayed inputs.  Both go through
// v_mfma_f32_16x16x32_f16 over 16 chunks at a time, each operand split into
// an fp16 high part and the fp16 rounding of the remainder (hi*hi + hi*lo +
// lo*hi, FP32 accumulation; the coefficients scaled by a power of two that
// keeps them in the fp16 range).  The vector units carry the states from
// chunk to chunk, Y[c+1] = a^8 Y[c] + sum_s b a^(7-s) x[8c + s - d], with the
// carry correction of the per-sample form applied every C/8 chunks.
//
// One workgroup of 256 threads per (template, up to 256 of its filters);
// thread i runs the chunk chain of filter i, wave w owns filters
// 64w .. 64w+63 in the products.  The input window is staged once per
// sub-block already split, as fp16 high and low parts, each held twice (the
// second copy one sample ahead) so that 8 samples from any position are four
// aligned 32-bit reads.  Per 128-sample tile: the chain stores the 16 chunk
// states (scaled, split) in LDS; each wave multiplies its filters' blocks;
// the four waves' partial sums are added in LDS and written as the piece's
// band output.
// LDS: Xh0 Xh1 Xl0 Xl1 [xcap] fp16 each | Yh [16][kMfmaYRow] half2 | Yl [same] | zp [4][16][kMfmaZRow] f32
// (rows padded so that the 16 chunks of a column read, and the 4 row groups
// of a partial-sum store, fall in different banks)
// ---------------------------------------------------------------------------
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
constexpr int kMfmaK2 = 16;    // Toeplitz K-blocks per wave (4 filters x 8 samples each)
constexpr int kMfmaK1 = 4;     // state K-blocks per wave (16 filters x re/im each)
constexpr int kMfmaSP = 14;    // log2 scale of the powers a1^(t+1)
constexpr int kMfmaSY = 8;     // log2 scale of the chunk states
constexpr int kMfmaYRow = kMfmaSlots + 4;  // words per chunk row of the state tile
constexpr int kMfmaZRow = 17;              // words per row of a wave's partial sums

__device__ __forceinline__ void split16(float v, _Float16& hi, _Float16& lo)
{
    hi = (_Float16)v;
    lo = (_Float16)(v - (float)hi);
}

__device__ __forceinline__ uint32_t pack_h2(_Float16 a, _Float16 b)
{
    return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
}

// 8 fp16 values from position p of a window held twice (X1 one ahead of X0):
// four aligned 32-bit reads
__device__ __forceinline__ half8_t load8h(const _Float16* X0, const _Float16* X1, int p)
{
    const uint32_t* w = reinterpret_cast<const uint32_t*>((p & 1) ? X1 + p - 1 : X0 + p);
    const uint4 v = make_uint4(w[0], w[1], w[2], w[3]);
    return __builtin_bit_cast(half8_t, v);
}

__global__ void __launch_bounds__(kMfmaSlots, 2) k_filter_mfma(LaunchArgs args)
{
    extern __shared__ float sm[];
    const int bid = blockIdx.x;
    int lo = 0, hi = args.nseg;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (args.cum[mid] <= bid) lo = mid;
        else hi = mid;
    }
    const ReqArg& q = args.req[args.seg_req[lo]];
    CBankDev* bd = cmem(q.bd);
    const WgDesc wg = cmem(bd->wg)[bd->band_wg0[0] + (bid - args.cum[lo])];
    const PieceDesc pd = cmem(bd->piece)[wg.piece_base];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int n = q.n;
    const int64_t s0 = cmem(bd->clock)[0];
    const int xcap = bd->xcap;  // a multiple of 32 samples
    _Float16* Xh0 = reinterpret_cast<_Float16*>(sm);
    _Float16* Xh1 = Xh0 + xcap;
    _Float16* Xl0 = Xh1 + xcap;
    _Float16* Xl1 = Xl0 + xcap;
    uint32_t* Yh = reinterpret_cast<uint32_t*>(Xl1 + xcap);
    uint32_t* Yl = Yh + 16 * kMfmaYRow;
    float* zp = reinterpret_cast<float*>(Yl + 16 * kMfmaYRow);

    // chunk chain of filter slot tid
    const int64_t g = wg.slot_base + tid;
    const SPIIR_AS_CONST c32* kc = cmem(bd->kc);
    const SPIIR_AS_CONST c32* pw = cmem(bd->pw);
    c32 Y = gmem(bd->y)[g], u = gmem(bd->ys)[g];
    const c32 a8 = cmem(bd->a)[g], dc = cmem(bd->dc)[g];
    const int dA = cmem(bd->off)[g];
    float wr[kMfmaT], wi[kMfmaT];  // b a^(7-s): weight of sample s in the chunk's end state
#pragma unroll
    for (int s = 0; s < kMfmaT; ++s) {
        const c32 k = kc[g * kMfmaT + (kMfmaT - 1 - s)];
        wr[s] = k.x;
        wi[s] = k.y;
    }
    const int64_t cmask = bd->C - 1;

    // matrix operands of this wave: row r = (t, part), column group g4
    const int r = lane & 15, g4 = lane >> 4, t = r & 7, part = r >> 3, col = lane & 15;
    const float sA = ldexpf(1.0f, wg.scale);
    half8_t Ah[kMfmaK2], Al[kMfmaK2], Ph[kMfmaK1], Pl[kMfmaK1];
    int dB[kMfmaK2];
#pragma unroll
    for (int kb = 0; kb < kMfmaK2; ++kb) {
        const int64_t gf = wg.slot_base + wave * 64 + 4 * kb + g4;
#pragma unroll
        for (int s = 0; s < kMfmaT; ++s) {
            const c32 k = kc[gf * kMfmaT + ((t - s) & (kMfmaT - 1))];
            const float v = s <= t ? (part ? k.y : k.x) * sA : 0.0f;
            _Float16 h, l;
            split16(v, h, l);
            Ah[kb][s] = h;
            Al[kb][s] = l;
        }
        dB[kb] = cmem(bd->off)[gf];
    }
#pragma unroll
    for (int kb = 0; kb < kMfmaK1; ++kb) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t gf = wg.slot_base + wave * 64 + 16 * kb + 4 * g4 + (j >> 1);
            const c32 p = pw[gf * kMfmaT + t];
            // row (t, re): Re p Re Y - Im p Im Y;  row (t, im): Im p Re Y + Re p Im Y
            const float v = part == 0 ? ((j & 1) ? -p.y : p.x) : ((j & 1) ? p.x : p.y);
            _Float16 h, l;
            split16(ldexpf(v, kMfmaSP), h, l);
            Ph[kb][j] = h;
            Pl[kb][j] = l;
        }
    }
    const float unA = ldexpf(1.0f, -wg.scale), unP = ldexpf(1.0f, -(kMfmaSP + kMfmaSY));
    const float sY = ldexpf(1.0f, kMfmaSY);

    const int S = bd->S[0];
    const SPIIR_AS_CONST float* ring = cmem(bd->rings) + bd->ring_off[0];
    const int64_t mk = bd->ring_mask[0];
    SPIIR_AS_GLOBAL float* zout = reinterpret_cast<SPIIR_AS_GLOBAL float*>(gmem(q.zw) + pd.zoff);
    bool sat = false;
    for (int kb0 = 0; kb0 < n; kb0 += S) {
        const int sub = min(S, n - kb0);
        const int64_t origin = ((s0 + kb0 - wg.maxd - 1) >> 6) << 6;
        const int wn = (int)(s0 + kb0 + sub - origin);
        __syncthreads();
        // thread j writes word j of each copy: samples (2j, 2j+1) of X*0 and
        // (2j+1, 2j+2) of X*1, from x[origin + 2j .. origin + 2j + 2]
        uint32_t* Wh0 = reinterpret_cast<uint32_t*>(Xh0);
        uint32_t* Wh1 = reinterpret_cast<uint32_t*>(Xh1);
        uint32_t* Wl0 = reinterpret_cast<uint32_t*>(Xl0);
        uint32_t* Wl1 = reinterpret_cast<uint32_t*>(Xl1);
        for (int j = tid; 2 * j < wn; j += kMfmaSlots) {
            const int i = 2 * j;
            const float v0 = ring[(origin + i) & mk];
            const float v1 = i + 1 <= wn ? ring[(origin + i + 1) & mk] : 0.0f;
            const float v2 = i + 2 <= wn ? ring[(origin + i + 2) & mk] : 0.0f;
            _Float16 h0, l0, h1, l1, h2, l2;
            split16(v0, h0, l0);
            split16(v1, h1, l1);
            split16(v2, h2, l2);
            Wh0[j] = pack_h2(h0, h1);
            Wl0[j] = pack_h2(l0, l1);
            Wh1[j] = pack_h2(h1, h2);
            Wl1[j] = pack_h2(l1, l2);
        }
        __syncthreads();
        for (int k0 = kb0; k0 < kb0 + sub; k0 += kMfmaTile) {
            const int rel0 = (int)(s0 + k0 - origin);  // window position of the tile's first sample
            // chunk chain, four chunks at a time: their input sums first
            // (independent), then the states in order, each stored (scaled,
            // split) before its chunk
#pragma unroll 1
            for (int c4 = 0; c4 < 16; c4 += 4) {
            float er[4], ei[4];
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
                const int p = rel0 + kMfmaT * (c4 + cc) - dA;
                const half8_t xh = load8h(Xh0, Xh1, p);
                const half8_t xl = load8h(Xl0, Xl1, p);
                float ar = 0.0f, ai = 0.0f, br = 0.0f, bi = 0.0f;
#pragma unroll
                for (int s = 0; s < kMfmaT; ++s) {
                    const float x = (float)xh[s] + (float)xl[s];
                    if (s & 1) {
                        br = fmaf(wr[s], x, br);
                        bi = fmaf(wi[s], x, bi);
                    } else {
                        ar = fmaf(wr[s], x, ar);
                        ai = fmaf(wi[s], x, ai);
                    }
                }
                er[cc] = ar + br;
                ei[cc] = ai + bi;
            }
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
                const int c = c4 + cc;
                _Float16 hr, lr, hi_, li;
                const float yr = Y.x * sY, yi = Y.y * sY;
                sat |= !(fabsf(yr) < 32768.0f && fabsf(yi) < 32768.0f);
                split16(yr, hr, lr);
                split16(yi, hi_, li);
                Yh[c * kMfmaYRow + tid] = pack_h2(hr, hi_);
                Yl[c * kMfmaYRow + tid] = pack_h2(lr, li);
                const float nr = fmaf(a8.x, Y.x, fmaf(-a8.y, Y.y, er[cc]));
                const float ni = fmaf(a8.x, Y.y, fmaf(a8.y, Y.x, ei[cc]));
                Y = c32{nr, ni};
                if (((s0 + k0 + kMfmaT * (c + 1)) & cmask) == 0) {
                    Y.x += u.x;
                    Y.y += u.y;
                    u = c32{fmaf(dc.x, Y.x, -dc.y * Y.y), fmaf(dc.x, Y.y, dc.y * Y.x)};
                }
            }
            }
            __syncthreads();
            // the wave's filters: Toeplitz input part and state part of 16 chunks,
            // in independent accumulators
            f32x4_t D2[4], D1[2];
#pragma unroll
            for (int i = 0; i < 4; ++i) D2[i] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int i = 0; i < 2; ++i) D1[i] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kb = 0; kb < kMfmaK2; ++kb) {
                const int p = rel0 + kMfmaT * col - dB[kb];
                const half8_t bh = load8h(Xh0, Xh1, p);
                const half8_t bl = load8h(Xl0, Xl1, p);
                f32x4_t& D = D2[kb & 3];
                D = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ah[kb], bh, D, 0, 0, 0);
                D = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ah[kb], bl, D, 0, 0, 0);
                D = __builtin_amdgcn_mfma_f32_16x16x32_f16(Al[kb], bh, D, 0, 0, 0);
            }
#pragma unroll
            for (int kb = 0; kb < kMfmaK1; ++kb) {
                const int f0 = wave * 64 + 16 * kb + 4 * g4;
                const uint4 hv = *reinterpret_cast<const uint4*>(Yh + col * kMfmaYRow + f0);
                const uint4 lv = *reinterpret_cast<const uint4*>(Yl + col * kMfmaYRow + f0);
                const half8_t bh = __builtin_bit_cast(half8_t, hv);
                const half8_t bl = __builtin_bit_cast(half8_t, lv);
                f32x4_t& D = D1[kb & 1];
                D = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ph[kb], bh, D, 0, 0, 0);
                D = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ph[kb], bl, D, 0, 0, 0);
                D = __builtin_amdgcn_mfma_f32_16x16x32_f16(Pl[kb], bh, D, 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float v2 = (D2[0][i] + D2[1][i]) + (D2[2][i] + D2[3][i]);
                zp[(wave * 16 + 4 * g4 + i) * kMfmaZRow + col] = fmaf(v2, unA, (D1[0][i] + D1[1][i]) * unP);
            }
            __syncthreads();
            // sum of the four waves' partials: element (row, chunk) = (tid >> 4, tid & 15)
            {
                const int row = tid >> 4, ch = tid & 15;
                const float* zr = zp + row * kMfmaZRow + ch;
                const float v = (zr[0] + zr[16 * kMfmaZRow]) + (zr[32 * kMfmaZRow] + zr[48 * kMfmaZRow]);
                zout[2 * (int64_t)(k0 + kMfmaT * ch + (row & 7)) + (row >> 3)] = v;
            }
        }
    }
    gmem(bd->y)[g] = Y;
    gmem(bd->ys)[g] = u;
    if (sat || !(isfinite(Y.x) && isfinite(Y.y))) atomicOr(&bd->flags[pd.tmpl], 1);
}

// ---------------------------------------------------------------------------
// Upsample-and-add chain, one workgroup of kUpThreads per (request, template).
// The piece sums of bands 1.. are fetched into registers first (one burst of
// independent loads), band 0's once the lowest band is in LDS, so they arrive
// while the chain runs from LDS, lowest band first.  A thread owns low-rate
// samples m = tid + kUpThreads*i of acc_{h+1} and writes both polyphase
// outputs acc_h[2m] and acc_h[2m+1] from the same window.
// LDS: cur [hu_len + max_block/2] c32 | nxt [same] | histories of bands
// 1..H-2 [(H-2) hu_len] c32 | taps [tu]
// ---------------------------------------------------------------------------
constexpr int kUpThreads = 256;
constexpr int kUpFastTaps = 32;  // interpolator length with an unrolled path

// low-rate samples per thread for the boundary between band h and h+1
__host__ __device__ constexpr int up_slots(int h)
{
    return (kInnerBlock >> (h + 1)) / kUpThreads > 1 ? (kInnerBlock >> (h + 1)) / kUpThreads : 1;
}
__host__ __device__ constexpr int up_slot_base(int h)
{
    return h == 0 ? 0 : up_slot_base(h - 1) + up_slots(h - 1);
}
constexpr int kUpSlotsTotal = up_slot_base(kMaxBands);
// sample pairs (2m, 2m+1) of band h in a block of n base-rate samples
__device__ __forceinline__ int up_pairs(int n, int h) { return ((n >> h) + 1) >> 1; }

// Adds piece p of band h's segment to the thread's slots of pv (piece 0 is
// loaded into the zeroed slots, the others are added in piece order).
__device__ __forceinline__ void up_load(float4 (&pv)[kUpSlotsTotal], int h, const SPIIR_AS_CONST c32* zw,
                                        const SegDesc& sg, int64_t zstride, int n, int tid, int p)
{
    if (sg.npiece <= p) return;
    const SPIIR_AS_CONST float4* row =
        reinterpret_cast<const SPIIR_AS_CONST float4*>(zw + sg.zoff + p * zstride);
#pragma unroll
    for (int i = 0; i < up_slots(h); ++i) {
        const int m = tid + kUpThreads * i;
        if (m < up_pairs(n, h)) {
            const float4 u = row[m];
            float4& v = pv[up_slot_base(h) + i];
            if (p == 0) {
                v = u;
            } else {
                v.x += u.x;
                v.y += u.y;
                v.z += u.z;
                v.w += u.w;
            }
        }
    }
}

__device__ __forceinline__ c32 piece_sum(const SPIIR_AS_CONST c32* zw, const SegDesc& sg, int64_t stride, int k)
{
    float vr = 0.0f, vi = 0.0f;
    for (int p = 0; p < sg.npiece; ++p) {
        const c32 u = zw[sg.zoff + p * stride + k];
        vr += u.x;
        vi += u.y;
    }
    return c32{vr, vi};
}

// Trigger reduction of one template's block (the step after the filter in the
// search pipeline, §5): the largest |z|^2, the first sample attaining it and
// the number of samples at or above a threshold.  |z|^2 is re*re + im*im with
// each product and the sum rounded to FP32 (no contraction), so a caller can
// repeat the decision exactly from the FP32 output.
struct PeakAcc {
    float v = -1.0f;
    int i = INT_MAX;
    int cnt = 0;
    __device__ __forceinline__ void add(float re, float im, int k, float thr2)
    {
#pragma clang fp contract(off)
        const float m = re * re + im * im;  // two rounded products, one rounded sum
        if (m > v) {  // a thread visits its samples in increasing order
            v = m;
            i = k;
        }
        cnt += m >= thr2 ? 1 : 0;
    }
    __device__ __forceinline__ void merge(float ov, int oi, int oc)
    {
        if (ov > v || (ov == v && oi < i)) {
            v = ov;
            i = oi;
        }
        cnt += oc;
    }
};

// `lds`: 12 words of the kernel's dynamic LDS that no thread reads any more
// (the kernel keeps no static LDS, so its dynamic limit can be raised to the
// full 160 KB).
__device__ void peak_store(PeakAcc a, const ReqArg& q, int t, int tid, float* lds)
{
    float* sv = lds;
    int* si = reinterpret_cast<int*>(lds + kUpThreads / 64);
    int* sc = si + kUpThreads / 64;
    for (int off = 32; off >= 1; off >>= 1)
        a.merge(__shfl_xor(a.v, off), __shfl_xor(a.i, off), __shfl_xor(a.cnt, off));
    if ((tid & 63) == 0) {
        sv[tid >> 6] = a.v;
        si[tid >> 6] = a.i;
        sc[tid >> 6] = a.cnt;
    }
    __syncthreads();
    if (tid != 0) return;
    for (int w = 1; w < kUpThreads / 64; ++w) a.merge(sv[w], si[w], sc[w]);
    SPIIR_AS_GLOBAL spiir_peak* pk = gmem(q.peaks) + t;
    float v = a.v;
    int idx = a.i == INT_MAX ? -1 : q.c0 + a.i;
    int cnt = a.cnt;
    if (q.c0 > 0) {  // later chunk of the caller's block: combine with the earlier ones
        const spiir_peak old = *pk;
        if (!(idx >= 0 && (old.index < 0 || v > old.peak2))) {
            v = old.peak2;
            idx = old.index;
        }
        cnt += old.n_above;
    }
    *pk = spiir_peak{v, idx, cnt, 0};
}

__global__ void __launch_bounds__(kUpThreads, 4) k_upadd(LaunchArgs args)
{
    extern __shared__ float sm[];
    const int bid = blockIdx.x;
    int r = 0;
    while (r + 1 < args.nreq && args.tcum[r + 1] <= bid) ++r;
    const ReqArg& q = args.req[r];
    CBankDev* bd = cmem(q.bd);
    const int t = bid - args.tcum[r];
    const int tid = threadIdx.x;
    const int H = bd->H, n = q.n, HU = bd->hu_len, tu = bd->tu, MB = bd->max_block;
    const SPIIR_AS_CONST SegDesc* seg = cmem(bd->seg) + (int64_t)t * H;
    const SPIIR_AS_CONST c32* zw = cmem(q.zw);
    SPIIR_AS_GLOBAL c32* zrow = q.z ? gmem(q.z) + (int64_t)t * q.ldz : nullptr;
    const bool peaks = q.peaks != nullptr;
    PeakAcc acc;
    // The common 32-tap interpolator reads its taps as uniform scalar loads
    // and runs the tap loop unrolled; other lengths read the taps from LDS.
    // Both add the terms in the same order, so they give the same bits.
    const bool taps32 = tu == kUpFastTaps;
    const SPIIR_AS_CONST float* tap = cmem(bd->hu);

    if (H == 1) {
        const SegDesc sg = seg[0];
        for (int k = tid; k < n; k += kUpThreads) {
            const c32 v = piece_sum(zw, sg, bd->zstride[0], k);
            if (zrow) zrow[k] = v;
            if (peaks) acc.add(v.x, v.y, k, q.thr2);
        }
        if (peaks) peak_store(acc, q, t, tid, sm);  // this path uses no other LDS
        return;
    }

    const int ext = HU + MB / 2;
    c32* cur = reinterpret_cast<c32*>(sm);
    c32* nxt = cur + ext;
    c32* hl = nxt + ext;  // histories of bands 1..H-2, loaded once up front
    float* hu = reinterpret_cast<float*>(hl + (H - 2) * HU);
    for (int i = tid; i < tu; i += kUpThreads) hu[i] = tap[i];
    const SPIIR_AS_GLOBAL c32* hist_in = gmem(bd->uphist) + ((int64_t)t * H + 1) * HU;
    for (int i = tid; i < (H - 2) * HU; i += kUpThreads) hl[i] = hist_in[i];

    // Every band's own output, as sample pairs (2m, 2m+1) (the lowest band may
    // end on an unpaired sample; its partner is a workspace word that is read
    // but not used).  Bands 1.. are loaded for all slots at once (independent
    // loads, one wait), then the other pieces of split segments are added.
    // Band 0, the largest, is loaded once the lowest band is in place, so its
    // loads are in flight while the chain runs through the lower bands.
    float4 pv[kUpSlotsTotal];
#pragma unroll
    for (int h = 0; h < kMaxBands; ++h)
#pragma unroll
        for (int i = 0; i < up_slots(h); ++i) pv[up_slot_base(h) + i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int h = 1; h < kMaxBands; ++h)
        if (h < H) up_load(pv, h, zw, seg[h], bd->zstride[h], n, tid, 0);
#pragma unroll
    for (int h = 1; h < kMaxBands; ++h) {
        if (h >= H) continue;
        const SegDesc sg = seg[h];
        for (int p = 1; p < sg.npiece; ++p) up_load(pv, h, zw, sg, bd->zstride[h], n, tid, p);
    }

    // lowest band: acc_{H-1} = z_{H-1}, placed after its history
    {
        const int nh = n >> (H - 1);
        SPIIR_AS_GLOBAL c32* hist = gmem(bd->uphist) + ((int64_t)t * H + H - 1) * HU;
        for (int i = tid; i < HU; i += kUpThreads) cur[i] = hist[i];
#pragma unroll
        for (int h = 1; h < kMaxBands; ++h) {
            if (h == H - 1) {
#pragma unroll
                for (int i = 0; i < up_slots(h); ++i) {
                    const int m = tid + kUpThreads * i;
                    if (m < up_pairs(n, h)) {
                        const float4 v = pv[up_slot_base(h) + i];
                        cur[HU + 2 * m] = c32{v.x, v.y};
                        if (2 * m + 1 < nh) cur[HU + 2 * m + 1] = c32{v.z, v.w};
                    }
                }
            }
        }
        __syncthreads();
        for (int i = tid; i < HU; i += kUpThreads) hist[i] = cur[nh + i];
    }
    up_load(pv, 0, zw, seg[0], bd->zstride[0], n, tid, 0);

    const int ne = HU, no = tu / 2;  // even and odd polyphase tap counts
#pragma unroll
    for (int h = kMaxBands - 2; h >= 0; --h) {
        if (h <= H - 2) {
            const int nh = n >> h, nlo = n >> (h + 1);
            SPIIR_AS_GLOBAL c32* hist = gmem(bd->uphist) + ((int64_t)t * H + h) * HU;
            if (h > 0)
                for (int i = tid; i < HU; i += kUpThreads) nxt[i] = hl[(h - 1) * HU + i];
            if (h == 0)
                for (int p = 1; p < seg[0].npiece; ++p) up_load(pv, 0, zw, seg[0], bd->zstride[0], n, tid, p);
            // all of the thread's slots hold samples of this block
            const bool full = nlo >= kUpThreads * up_slots(h);
#pragma unroll
            for (int i = 0; i < up_slots(h); ++i) {
                const int m = tid + kUpThreads * i;
                if (full || m < nlo) {
                    const float4 v = pv[up_slot_base(h) + i];
                    float er = v.x, ei = v.y, orr = v.z, oi = v.w;
                    const c32* a = cur + HU + m;
                    if (taps32) {
                        // the whole window first (independent LDS reads), then the taps
                        c32 u[kUpFastTaps / 2];
#pragma unroll
                        for (int j = 0; j < kUpFastTaps / 2; ++j) u[j] = a[-j];
#pragma unroll
                        for (int j = 0; j < kUpFastTaps / 2; ++j) {
                            er = fmaf(tap[2 * j], u[j].x, er);
                            ei = fmaf(tap[2 * j], u[j].y, ei);
                            orr = fmaf(tap[2 * j + 1], u[j].x, orr);
                            oi = fmaf(tap[2 * j + 1], u[j].y, oi);
                        }
                    } else {
                        for (int j = 0; j < ne; ++j) {
                            const c32 u = a[-j];
                            const float ce = hu[2 * j];
                            er = fmaf(ce, u.x, er);
                            ei = fmaf(ce, u.y, ei);
                            if (j < no) {
                                const float co = hu[2 * j + 1];
                                orr = fmaf(co, u.x, orr);
                                oi = fmaf(co, u.y, oi);
                            }
                        }
                    }
                    if (h == 0) {
                        if (zrow) {
                            zrow[2 * m] = c32{er, ei};
                            zrow[2 * m + 1] = c32{orr, oi};
                        }
                        if (peaks) {
                            acc.add(er, ei, 2 * m, q.thr2);
                            acc.add(orr, oi, 2 * m + 1, q.thr2);
                        }
                    } else {
                        nxt[HU + 2 * m] = c32{er, ei};
                        nxt[HU + 2 * m + 1] = c32{orr, oi};
                    }
                }
            }
            __syncthreads();
            if (h > 0) {
                for (int i = tid; i < HU; i += kUpThreads) hist[i] = nxt[nh + i];
                c32* tmp = cur;
                cur = nxt;
                nxt = tmp;
            }
        }
    }
    if (peaks) peak_store(acc, q, t, tid, sm);  // after the last phase's barrier
}

// ---------------------------------------------------------------------------
// Time split, middle pass: per filter slot, the start state of every chunk
// after the first, S[c+1] = uend[c] + a1^lc S[c] with S[first+1] = uend[first]
// (the first chunk's end state, which ran from the carried state).  The
// product uses the same component formula as the recurrence, so it also holds
// for the swapped form of odd lanes.  One thread per slot; request r owns
// blocks [cum[r], cum[r+1]).
// ---------------------------------------------------------------------------
constexpr int kChainThreads = 256;

__global__ void __launch_bounds__(kChainThreads) k_chain(LaunchArgs args)
{
    const int bid = blockIdx.x;
    int r = 0;
    while (r + 1 < args.nreq && args.cum[r + 1] <= bid) ++r;
    const ReqArg& q = args.req[r];
    CBankDev* bd = cmem(q.bd);
    const int64_t g = (int64_t)(bid - args.cum[r]) * kChainThreads + threadIdx.x;
    if (g >= bd->n_slots) return;
    const int h = cmem(bd->wg)[g / ((int64_t)bd->F * bd->L)].band;
    const int nh = q.n >> h, lc = bd->lc[h];
    const int64_t s0h = cmem(bd->clock)[0] >> h;
    const int64_t B = (s0h + lc - 1) / lc * lc;
    const int first_c = B == s0h ? 1 : 0;
    const int last_c = s0h + nh - 1 < B ? 0 : 1 + (int)((s0h + nh - 1 - B) / lc);
    const int64_t ns = bd->n_slots;
    const SPIIR_AS_CONST c32* uend = cmem(bd->uend);
    SPIIR_AS_GLOBAL c32* schain = gmem(bd->schain);
    c32 st = uend[first_c * ns + g];
    const c32 al = cmem(bd->al)[g];
    for (int c = first_c + 1; c <= last_c; ++c) {
        schain[c * ns + g] = st;
        if (c < last_c) {
            const c32 u = uend[c * ns + g];
            st = c32{fmaf(al.x, st.x, fmaf(-al.y, st.y, u.x)), fmaf(al.x, st.y, fmaf(al.y, st.x, u.y))};
        }
    }
}

int launch_chain(const LaunchArgs& a, int64_t nblocks, void* stream)
{
    hipLaunchKernelGGL(k_chain, dim3((unsigned)nblocks), dim3(kChainThreads), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 carry precompute and FP32 conversion of the tables (once, at create).
// ---------------------------------------------------------------------------
__device__ __forceinline__ c64 cmul(c64 u, c64 v)
{
    return c64{u.x * v.x - u.y * v.y, u.x * v.y + u.y * v.x};
}

__global__ void k_prep(const c64* __restrict__ a, const c64* __restrict__ b, int64_t n, int C,
                       c32* fa, c32* fb, c32* fdc, const int32_t* __restrict__ slot_lc, c32* fal)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const c64 av = a[i], bv = b[i];
    const float ar = (float)av.x, ai = (float)av.y;
    const double tr = ar, ti = ai;  // fl32(a1) carried in FP64
    double pr = 1.0, pi = 0.0, qr = 1.0, qi = 0.0;
    for (int c = 0; c < C; ++c) {
        const double npr = pr * av.x - pi * av.y, npi = pr * av.y + pi * av.x;
        const double nqr = qr * tr - qi * ti, nqi = qr * ti + qi * tr;
        pr = npr; pi = npi;
        qr = nqr; qi = nqi;
    }
    const float dcr = (float)(pr - qr), dci = (float)(pi - qi);
    // a1^lc for the time split, by repeated squaring in FP64
    c64 al{1.0, 0.0};
    if (slot_lc) {
        c64 base = av;
        for (int e = slot_lc[i]; e > 0; e >>= 1) {
            if (e & 1) al = cmul(al, base);
            base = cmul(base, base);
        }
    }
    const float alr = (float)al.x, ali = (float)al.y;
    if (i & 1) {
        // odd lane (slots of a workgroup are lane-contiguous and L is even):
        // tables for the swapped state (Im y, Re y)
        fa[i] = c32{ar, -ai};
        fb[i] = c32{(float)bv.y, (float)bv.x};
        fdc[i] = c32{dcr, -dci};
        if (fal) fal[i] = c32{alr, -ali};
    } else {
        fa[i] = c32{ar, ai};
        fb[i] = c32{(float)bv.x, (float)bv.y};
        fdc[i] = c32{dcr, dci};
        if (fal) fal[i] = c32{alr, ali};
    }
}

__global__ void k_fill(uint32_t* p, int64_t words)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
int launch_stage(const LaunchArgs& a, int lds_bytes, void* stream)
{
    hipLaunchKernelGGL(k_stage, dim3(a.nreq), dim3(kStageThreads), lds_bytes, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

template <int F, bool COMP, bool LOCAL>
static int launch_filter_t(const LaunchArgs& a, int nblocks, int L, int lds_bytes,
                           hipStream_t s)
{
    hipLaunchKernelGGL((k_filter<F, COMP, LOCAL>), dim3(nblocks), dim3(L), lds_bytes, s, a);
    return (int)hipGetLastError();
}

template <int F, bool COMP>
static int allow_lds_t()
{
    int e = (int)hipFuncSetAttribute((const void*)k_filter<F, COMP, false>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, filter_max_lds());
    if (!e)
        e = (int)hipFuncSetAttribute((const void*)k_filter<F, COMP, true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, filter_max_lds());
    return e;
}

// Raises the dynamic LDS limit of the filter-kernel variants and the
// upsample-and-add kernel on the current device (done outside any launch
// sequence, so recorded sequences hold launches only).
int allow_filter_lds()
{
    int e = (int)hipFuncSetAttribute((const void*)k_upadd, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     filter_max_lds());
    if (!e)
        e = (int)hipFuncSetAttribute((const void*)k_filter_mfma, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     filter_max_lds());
    if (!e) e = allow_lds_t<1, false>();
    if (!e) e = allow_lds_t<1, true>();
    if (!e) e = allow_lds_t<2, false>();
    if (!e) e = allow_lds_t<2, true>();
    if (!e) e = allow_lds_t<4, false>();
    if (!e) e = allow_lds_t<4, true>();
    if (!e) e = allow_lds_t<6, false>();
    if (!e) e = allow_lds_t<6, true>();
    if (!e) e = allow_lds_t<8, false>();
    if (!e) e = allow_lds_t<8, true>();
    return e;
}

template <bool LOCAL>
static int launch_filter_any(int F, int precision, const LaunchArgs& a, int nblocks, int L,
                             int lds_bytes, hipStream_t s)
{
    const bool comp = precision == SPIIR_FP32_COMPENSATED;
    switch (F) {
    case 1: return comp ? launch_filter_t<1, true, LOCAL>(a, nblocks, L, lds_bytes, s)
                        : launch_filter_t<1, false, LOCAL>(a, nblocks, L, lds_bytes, s);
    case 2: return comp ? launch_filter_t<2, true, LOCAL>(a, nblocks, L, lds_bytes, s)
                        : launch_filter_t<2, false, LOCAL>(a, nblocks, L, lds_bytes, s);
    case 4: return comp ? launch_filter_t<4, true, LOCAL>(a, nblocks, L, lds_bytes, s)
                        : launch_filter_t<4, false, LOCAL>(a, nblocks, L, lds_bytes, s);
    case 6: return comp ? launch_filter_t<6, true, LOCAL>(a, nblocks, L, lds_bytes, s)
                        : launch_filter_t<6, false, LOCAL>(a, nblocks, L, lds_bytes, s);
    case 8: return comp ? launch_filter_t<8, true, LOCAL>(a, nblocks, L, lds_bytes, s)
                        : launch_filter_t<8, false, LOCAL>(a, nblocks, L, lds_bytes, s);
    default: return (int)hipErrorInvalidValue;
    }
}

int launch_filter(int F, int precision, const LaunchArgs& a, int nblocks, int L, int lds_bytes,
                  void* stream)
{
    return launch_filter_any<false>(F, precision, a, nblocks, L, lds_bytes, (hipStream_t)stream);
}

// the end-state pass of a time split (the compensated sum plays no part in it)
int launch_filter_local(int F, int precision, const LaunchArgs& a, int nblocks, int L, int lds_bytes,
                        void* stream)
{
    (void)precision;
    return launch_filter_any<true>(F, SPIIR_FP32, a, nblocks, L, lds_bytes, (hipStream_t)stream);
}

int launch_filter_mfma(const LaunchArgs& a, int nblocks, int lds_bytes, void* stream)
{
    hipLaunchKernelGGL(k_filter_mfma, dim3(nblocks), dim3(kMfmaSlots), lds_bytes, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_upadd(const LaunchArgs& a, int nblocks, int lds_bytes, void* stream)
{
    hipLaunchKernelGGL(k_upadd, dim3(nblocks), dim3(kUpThreads), lds_bytes, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_prep(const c64* a, const c64* b, int64_t n, int C, c32* fa, c32* fb, c32* fdc,
                const int32_t* slot_lc, c32* fal, void* stream)
{
    if (n <= 0) return 0;
    const int bs = 256;
    const int64_t nb = (n + bs - 1) / bs;
    hipLaunchKernelGGL(k_prep, dim3((unsigned)nb), dim3(bs), 0, (hipStream_t)stream, a, b, n, C,
                       fa, fb, fdc, slot_lc, fal);
    return (int)hipGetLastError();
}

int launch_fill(void* p, int64_t bytes, void* stream)
{
    if (bytes <= 0) return 0;
    const int64_t words = bytes / 4;
    int64_t nb = (words + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)nb), dim3(256), 0, (hipStream_t)stream,
                       (uint32_t*)p, words);
    return (int)hipGetLastError();
}

int filter_max_lds() { return 160 * 1024; }

// ---------------------------------------------------------------------------
// Static workspace of spiir_process_block_noalloc: one array per device,
// loaded with the code object and held until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is a stand-in,
// not a device address); it passes the address hipGetSymbolAddress returns
// for the current device, taken once per device and kept.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;

int scratch_ptr(int device, void** out)
{
    static std::mutex mu;
    static void* ptrs[kMaxDevices] = {};
    *out = nullptr;
    int cur = -1;
    if (device < 0 || device >= kMaxDevices) return (int)hipErrorInvalidDevice;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return (int)e;
    if (cur != device) return (int)hipErrorInvalidDevice;  // the device must be current
    std::lock_guard<std::mutex> lk(mu);
    if (!ptrs[device]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        if (!p) return (int)hipErrorInvalidSymbol;
        ptrs[device] = p;
    }
    *out = ptrs[device];
    return 0;
}

}  // namespace spiir
