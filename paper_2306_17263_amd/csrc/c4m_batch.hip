// c4m_batch.hip -- batched form: many independent 2D TM cavity problems of
// uneven N advanced together.
//
// A step is four stages per problem: the Step 1 x-lines (XE), the Step 1
// solve (CE), the Step 2 x-lines (XH) and the Step 2 Hx and Hy solves (CH).
// Each stage is a table of work items (problem, item within the problem)
// over every problem; workgroups take items from per-XCD chunks of a table
// (their own XCD's chunk first), so problems of very different sizes share
// the machine.
//
// Strip form (FP64, the default): ONE persistent launch per step.  A
// workgroup works through the stages in order; an item of stage s of
// problem p first waits until every stage s-1 item of p has finished
// (per-problem counters, agent-scope release before a count moves and
// acquire after it is seen), so the stages of different problems overlap
// instead of meeting at launch boundaries.  Every workgroup of the grid is
// resident at once (grid = occupancy), items of a stage are only taken once
// the previous stage's table is exhausted, and every wait is bounded (it
// gives up after a poll limit and sets a sticky error flag), so the launch
// always drains.  The n-step loop is captured once as a HIP graph of
// launches and replayed.
// Column-tile form (tile_x 1-3, FP32-refined): one persistent launch per
// stage (the Step 2 Hx and Hy solves separately).
#include <hip/hip_runtime.h>
#include <string.h>

#include <math.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "c4m_stream_2d.h"

namespace c4m {

bool strip_form_2d(int shape, bool mixed, int sweeps);

// x-line items (one tile, or one band-table row) a workgroup takes at once
constexpr int X_TAKE = 8;

// Strip shape of the batched form: the single-problem default (8 steps per
// unrolled block, one step of prefetch, three waves per SIMD); the members'
// results do not depend on their segmentation, so they equal the problems
// run alone bit for bit.
constexpr int BS_U = 8, BS_LA = 1, BS_WPE = 3;

// stages; the column-tile form splits CH into its Hx and Hy launches
enum { ST_XE = 0, ST_CE = 1, ST_XH = 2, ST_CH = 3, ST_CHY = 4, NSTMAX = 5 };

struct BatchProb {
    XArgs xe, xh;            // x-line arguments of Step 1 and Step 2
    ColArgs ce, chx, chy;    // solve arguments
    int xe_tx, xe_tiles;     // Step 1 x-lines: tiles along x, tiles (band items follow)
    int xh_tx, xh_tiles;     // Step 2 x-lines
    int ce_ty, chx_ty, chy_ty;   // column-tile form: tiles along y of each solve
    int n_chx;               // strip form, stage CH: items of the Hx part (the Hy items follow)
    int items[NSTMAX];       // work items of each stage
    StripPlan plan[3];       // strip form: plans of the E, Hx and Hy solves
};

// One work item: problem index and item within the problem's stage.
struct Item {
    int p, local;
};

struct Stage {
    const Item* items;
    int total;
    int* ctr;                // [NXCD]: next item of each chunk
};

struct Sched {
    Stage st[NSTMAX];
    int* done;               // [count][NSTMAX]: items finished per problem and stage
    int* finished;           // workgroups that left the launch
    int* err;                // sticky: a stage wait gave up
    int count;
    int wait_limit;          // polls before a stage wait gives up
};

// Take up to `take` consecutive items of a stage for the workgroup (called
// by one thread; the atomics on a chunk counter are serialised, so small
// items are taken in runs): the item sequence is cut into NXCD contiguous
// chunks with one counter each; workgroup IDs are dealt to the XCDs in turn, so a
// workgroup takes items from the chunk of its XCD first and from the others
// once that is empty.  False when every chunk is exhausted.
__device__ __forceinline__ bool claim_items(const Stage& q, int take, int& first, int& cnt)
{
    const int per = (q.total + NXCD - 1) / NXCD;
    const int home = (int)(blockIdx.x % NXCD);
    for (int j = 0; j < NXCD; ++j) {
        const int c = (home + j) % NXCD;
        const int len = min(per, q.total - c * per);
        if (len <= 0) continue;
        const int k = atomicAdd(q.ctr + c, take);
        if (k < len) {
            first = c * per + k;
            cnt = min(take, len - k);
            return true;
        }
    }
    return false;
}

template <int K, int MODE>
__device__ __forceinline__ void batch_strip(const ColArgs& ca, const PadeLine& L, const StripPlan& plan, int local,
                                            const Coef& cf, const ChebSchedule& cs)
{
    using SS = StripShape<K, MODE, BS_U, BS_LA>;
    int strip, y0, tr;
    bool up;
    plan.item(local, strip, y0, tr, up);
    strip_tile<K, MODE, BS_U, BS_LA>(ca, cf, L, cs, ca.g.lo[0] + strip * SS::OW, y0, tr, up);
}

// band-table item `id` of an x-line stage: one thread per stored column of
// one band row at one end of the y-lines of the following solve
template <bool SPLIT>
__device__ __forceinline__ void batch_band(const ColArgs& ca, const XArgs& xa, int id)
{
    const int nbx = (xa.N + 1 + 255) / 256, nbr = band_rows(xa.L);
    const int gx = (id % nbx) * 256 + (int)threadIdx.x, r = (id / nbx) % nbr, e = id / (nbx * nbr);
    yband_entry<SPLIT>(ca.src, ca.yb, xa.N, xa.P, xa.L, gx, r, e);
}

// ---------------------------------------------------------------------------
// Strip form: one launch per step.
// ---------------------------------------------------------------------------
template <int K, bool TRACKED>
__global__ __launch_bounds__(SW_COLS * SW_WAVES) __attribute__((amdgpu_waves_per_eu(BS_WPE))) void k_batch_step(
    const BatchProb* __restrict__ bp, Sched sc, Coef cf, PadeTaps taps_xh, ChebSchedule cs)
{
    __shared__ double lds[XE_LDS > xt_lds(XL_H_TRACKED) ? XE_LDS : xt_lds(XL_H_TRACKED)];
    __shared__ int sl[4];
    constexpr int ME = TRACKED ? COL_E_TRACKED : COL_E_DISCRETE;
    constexpr int MHX = TRACKED ? COL_HX_TRACKED : COL_HX_DISCRETE;
    constexpr int MXH = TRACKED ? XL_H_TRACKED : XL_H_DISCRETE;
    const int tid = (int)threadIdx.x;
    int stage = 0;                       // thread 0: stage being taken
    for (;;) {
        __syncthreads();                 // the previous item's LDS and slot reads are done
        if (tid == 0) {
            int first = -1, cnt = 0;
            while (stage < ST_CH + 1) {
                const int take = (stage == ST_CE || stage == ST_CH) ? SW_WAVES : X_TAKE;
                if (claim_items(sc.st[stage], take, first, cnt)) break;
                ++stage;
            }
            if (first >= 0 && stage > 0) {
                // wait until the previous stage of each item's problem is done
                int prev = -1;
                for (int i = 0; i < cnt; ++i) {
                    const int p = sc.st[stage].items[first + i].p;
                    if (p == prev) continue;
                    prev = p;
                    const int need = bp[p].items[stage - 1];
                    const int* d = sc.done + p * NSTMAX + (stage - 1);
                    // bounded: after wait_limit polls, or once any wait of
                    // the launch has given up, stop waiting and flag it
                    int polls = 0;
                    while (__hip_atomic_load(d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                        if (++polls > sc.wait_limit ||
                            __hip_atomic_load(sc.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                            atomicOr(sc.err, 1);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                __threadfence();         // acquire: their results are visible from here on
            }
            sl[0] = stage;
            sl[1] = first;
            sl[2] = cnt;
        }
        __syncthreads();
        const int stg = sl[0], first = sl[1], cnt = sl[2];
        if (first < 0) break;
        if (stg == ST_XE || stg == ST_XH) {
            for (int i = 0; i < cnt; ++i) {
                if (i) __syncthreads();  // the previous tile's LDS reads are done
                const Item it = sc.st[stg].items[first + i];
                const BatchProb& B = bp[it.p];
                if (stg == ST_XE) {
                    if (it.local >= B.xe_tiles)
                        batch_band<true>(B.ce, B.xe, it.local - B.xe_tiles);
                    else
                        xlines_e_tile<TRACKED, true>(B.xe.src, B.xe.t0, B.xe.t1, B.xe.N, B.xe.P, B.xe.L, cf,
                                                     it.local % B.xe_tx, it.local / B.xe_tx, lds);
                } else {
                    if (it.local >= B.xh_tiles)
                        batch_band<!TRACKED>(B.chx, B.xh, it.local - B.xh_tiles);
                    else
                        xlines_tile<MXH>(B.xh.src, B.xh.t0, B.xh.t1, B.xh.N, B.xh.P, B.xh.L, cf, taps_xh,
                                         it.local % B.xh_tx, it.local / B.xh_tx, lds);
                }
            }
        } else {
            // strip items: one per wave
            const int w = __builtin_amdgcn_readfirstlane(tid / SW_COLS);
            if (w < cnt) {
                const Item it = sc.st[stg].items[first + w];
                const int p = __builtin_amdgcn_readfirstlane(it.p);
                const int local = __builtin_amdgcn_readfirstlane(it.local);
                const BatchProb& B = bp[p];
                if (stg == ST_CE)
                    batch_strip<K, ME>(B.ce, B.xe.L, B.plan[0], local, cf, cs);
                else if (local < B.n_chx)
                    batch_strip<K, MHX>(B.chx, B.xh.L, B.plan[1], local, cf, cs);
                else
                    batch_strip<K, COL_HY>(B.chy, B.xh.L, B.plan[2], local - B.n_chx, cf, cs);
            }
        }
        if (stg == ST_CH) continue;      // nothing waits on the last stage within the launch
        __syncthreads();
        if (tid == 0) {
            __threadfence();             // release: the items' results before their counts
            int prev = -1, add = 0;
            for (int i = 0; i < cnt; ++i) {
                const int p = sc.st[stg].items[first + i].p;
                if (p != prev && add) {
                    atomicAdd(sc.done + prev * NSTMAX + stg, add);
                    add = 0;
                }
                prev = p;
                ++add;
            }
            if (add) atomicAdd(sc.done + prev * NSTMAX + stg, add);
        }
    }
    // the last workgroup to leave resets every counter for the next launch
    if (tid == 0) {
        __threadfence();
        sl[3] = atomicAdd(sc.finished, 1) == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (sl[3]) {
        for (int i = tid; i < sc.count * NSTMAX; i += (int)blockDim.x) sc.done[i] = 0;
        if (tid < NSTMAX * NXCD) sc.st[tid / NXCD].ctr[tid % NXCD] = 0;
        __syncthreads();
        if (tid == 0) {
            *sc.finished = 0;
            __threadfence();
        }
    }
}

// ---------------------------------------------------------------------------
// Column-tile form: one persistent launch per stage.
// ---------------------------------------------------------------------------
// The last workgroup to leave resets the stage's chunk counters.
__device__ __forceinline__ void stage_finish(const Sched& sc, int stage)
{
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(sc.finished, 1) == (int)gridDim.x - 1) {
            for (int c = 0; c < NXCD; ++c) atomicExch(sc.st[stage].ctr + c, 0);
            atomicExch(sc.finished, 0);
        }
    }
}

// A run of up to `take` items for the workgroup: [slot[0], slot[0] + slot[1]).
// The same stages as separate launches (STAGE fixed): the launch boundary
// orders the stages, so there are no waits or counts.
// waves per SIMD each stage launch is compiled for: the strips need the
// registers of three; the Step 1 x-line tiles fit four workgroups in the
// LDS (the Step 2 tiles spill registers at five and run slower)
constexpr int stage_wpe(int st) { return st == ST_XE ? 4 : BS_WPE; }

template <int K, bool TRACKED, int STAGE>
__global__ __launch_bounds__(SW_COLS * SW_WAVES) __attribute__((amdgpu_waves_per_eu(stage_wpe(STAGE)))) void k_batch_stage(
    const BatchProb* __restrict__ bp, Sched sc, Coef cf, PadeTaps taps_xh, ChebSchedule cs)
{
    constexpr bool XL = STAGE == ST_XE || STAGE == ST_XH;
    __shared__ double lds[XL ? (STAGE == ST_XE ? XE_LDS : xt_lds(XL_H_TRACKED)) : 1];
    __shared__ int sl[2];
    constexpr int ME = TRACKED ? COL_E_TRACKED : COL_E_DISCRETE;
    constexpr int MHX = TRACKED ? COL_HX_TRACKED : COL_HX_DISCRETE;
    constexpr int MXH = TRACKED ? XL_H_TRACKED : XL_H_DISCRETE;
    const int tid = (int)threadIdx.x;
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            int first = -1, cnt = 0;
            sl[0] = claim_items(sc.st[STAGE], XL ? X_TAKE : SW_WAVES, first, cnt) ? first : -1;
            sl[1] = cnt;
        }
        __syncthreads();
        const int first = sl[0], cnt = sl[1];
        if (first < 0) break;
        if constexpr (XL) {
            for (int i = 0; i < cnt; ++i) {
                if (i) __syncthreads();
                const Item it = sc.st[STAGE].items[first + i];
                const BatchProb& B = bp[it.p];
                if constexpr (STAGE == ST_XE) {
                    if (it.local >= B.xe_tiles)
                        batch_band<true>(B.ce, B.xe, it.local - B.xe_tiles);
                    else
                        xlines_e_tile<TRACKED, true>(B.xe.src, B.xe.t0, B.xe.t1, B.xe.N, B.xe.P, B.xe.L, cf,
                                                     it.local % B.xe_tx, it.local / B.xe_tx, lds);
                } else {
                    if (it.local >= B.xh_tiles)
                        batch_band<!TRACKED>(B.chx, B.xh, it.local - B.xh_tiles);
                    else
                        xlines_tile<MXH>(B.xh.src, B.xh.t0, B.xh.t1, B.xh.N, B.xh.P, B.xh.L, cf, taps_xh,
                                         it.local % B.xh_tx, it.local / B.xh_tx, lds);
                }
            }
        } else {
            const int w = __builtin_amdgcn_readfirstlane(tid / SW_COLS);
            if (w < cnt) {
                const Item it = sc.st[STAGE].items[first + w];
                const int p = __builtin_amdgcn_readfirstlane(it.p);
                const int local = __builtin_amdgcn_readfirstlane(it.local);
                const BatchProb& B = bp[p];
                if constexpr (STAGE == ST_CE)
                    batch_strip<K, ME>(B.ce, B.xe.L, B.plan[0], local, cf, cs);
                else if (local < B.n_chx)
                    batch_strip<K, MHX>(B.chx, B.xh.L, B.plan[1], local, cf, cs);
                else
                    batch_strip<K, COL_HY>(B.chy, B.xh.L, B.plan[2], local - B.n_chx, cf, cs);
            }
        }
    }
    stage_finish(sc, STAGE);
}

// The x-line stages as plain grids: one workgroup per item, no claims.
// Workgroup IDs are dealt to the XCDs in turn, so workgroup b runs item
// (b mod 8) per + b / 8: every XCD walks one contiguous range of the table
// (a member's tiles together), in order.
template <bool TRACKED, int STAGE>
__global__ __launch_bounds__(SW_COLS * SW_WAVES) __attribute__((amdgpu_waves_per_eu(stage_wpe(STAGE)))) void k_batch_xstage(
    const BatchProb* __restrict__ bp, Sched sc, Coef cf, PadeTaps taps_xh)
{
    __shared__ double lds[STAGE == ST_XE ? XE_LDS : xt_lds(XL_H_TRACKED)];
    constexpr int MXH = TRACKED ? XL_H_TRACKED : XL_H_DISCRETE;
    const int n = sc.st[STAGE].total;
    const int per = (n + NXCD - 1) / NXCD;
    const int idx = (int)(blockIdx.x % NXCD) * per + (int)(blockIdx.x / NXCD);
    if (idx >= n) return;
    const Item it = sc.st[STAGE].items[idx];
    const BatchProb& B = bp[it.p];
    if constexpr (STAGE == ST_XE) {
        if (it.local >= B.xe_tiles)
            batch_band<true>(B.ce, B.xe, it.local - B.xe_tiles);
        else
            xlines_e_tile<TRACKED, true>(B.xe.src, B.xe.t0, B.xe.t1, B.xe.N, B.xe.P, B.xe.L, cf, it.local % B.xe_tx,
                                         it.local / B.xe_tx, lds);
    } else {
        if (it.local >= B.xh_tiles)
            batch_band<!TRACKED>(B.chx, B.xh, it.local - B.xh_tiles);
        else
            xlines_tile<MXH>(B.xh.src, B.xh.t0, B.xh.t1, B.xh.N, B.xh.P, B.xh.L, cf, taps_xh, it.local % B.xh_tx,
                             it.local / B.xh_tx, lds);
    }
}

__device__ __forceinline__ bool claim_run(const Sched& sc, int stage, int take, int* slot)
{
    __syncthreads();                     // every thread has read the previous items
    if (threadIdx.x == 0) {
        int first = -1, cnt = 0;
        slot[0] = claim_items(sc.st[stage], take, first, cnt) ? first : -1;
        slot[1] = cnt;
    }
    __syncthreads();
    return slot[0] >= 0;
}

template <int MODE>
__global__ __launch_bounds__(256) void k_batch_x(const BatchProb* __restrict__ bp, Sched sc, int stage, Coef cf,
                                                 PadeTaps taps)
{
    constexpr bool E = MODE == XL_E_TRACKED || MODE == XL_E_DISCRETE;
    __shared__ double lds[E ? XE_LDS : xt_lds(MODE)];
    __shared__ int slot[2];
    while (claim_run(sc, stage, X_TAKE, slot)) {
        for (int i = 0; i < slot[1]; ++i) {
            if (i) __syncthreads();
            const Item it = sc.st[stage].items[slot[0] + i];
            const BatchProb& B = bp[it.p];
            if constexpr (E)
                xlines_e_tile<MODE == XL_E_TRACKED, false>(B.xe.src, B.xe.t0, B.xe.t1, B.xe.N, B.xe.P, B.xe.L, cf,
                                                           it.local % B.xe_tx, it.local / B.xe_tx, lds);
            else
                xlines_tile<MODE>(B.xh.src, B.xh.t0, B.xh.t1, B.xh.N, B.xh.P, B.xh.L, cf, taps,
                                  it.local % B.xh_tx, it.local / B.xh_tx, lds);
        }
    }
    stage_finish(sc, stage);
}

template <int K, int MODE, class S, int FORM>
__global__ __launch_bounds__(S::NTC) __attribute__((amdgpu_waves_per_eu(S::NL == 4 ? 4 : 2))) void k_batch_col(
    const BatchProb* __restrict__ bp, Sched sc, int stage, Coef cf, PadeTaps taps, ChebSchedule cs)
{
    __shared__ int slot[2];
    while (claim_run(sc, stage, 2, slot)) {
        for (int i = 0; i < slot[1]; ++i) {
            if (i) __syncthreads();
            const Item it = sc.st[stage].items[slot[0] + i];
            const BatchProb& B = bp[it.p];
            const ColArgs& ca = stage == ST_CE ? B.ce : (stage == ST_CH ? B.chx : B.chy);
            const PadeLine& L = stage == ST_CE ? B.xe.L : B.xh.L;
            const int ty = stage == ST_CE ? B.ce_ty : (stage == ST_CH ? B.chx_ty : B.chy_ty);
            col_tile<K, MODE, S, FORM>(ca, cf, taps, L, cs, it.local / ty, it.local % ty);   // y fastest
        }
    }
    stage_finish(sc, stage);
}

// ---------------------------------------------------------------------------
// Host helpers: tile counts, occupancy, plans.
// ---------------------------------------------------------------------------
template <class F>
static auto with_k_bstrip(int K, F&& f)
{
    switch (K) {
        case 2: return f.template operator()<2>();
        case 3: return f.template operator()<3>();
        case 4: return f.template operator()<4>();
        case 5: return f.template operator()<5>();
        case 6: return f.template operator()<6>();
        case 7: return f.template operator()<7>();
        default: return f.template operator()<8>();
    }
}

static int col_tiles_k(int K, int shape, bool mixed, const UGrid& g, int* ty)
{
    if (mixed)
        return with_k_mixed(K, [&]<int KK, class S>() {
            *ty = col_tiles_y<KK, S>(g);
            return col_tiles_x<KK, S>(g) * col_tiles_y<KK, S>(g);
        });
    return with_k_shape(K, shape, [&]<int KK, class S>() {
        *ty = col_tiles_y<KK, S>(g);
        return col_tiles_x<KK, S>(g) * col_tiles_y<KK, S>(g);
    });
}

static int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) return 256;
    return cus;
}

// workgroups of a persistent launch: what fits on the device at once
template <class Kern>
static int resident_blocks(Kern kern, int threads)
{
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, threads, 0) != hipSuccess || per < 1) per = 1;
    return device_cus() * per;
}

template <int STAGE>
static int blocks_stage(int K, bool tracked)
{
    return with_k_bstrip(K, [&]<int KK>() {
        return tracked ? resident_blocks(k_batch_stage<KK, true, STAGE>, SW_COLS * SW_WAVES)
                       : resident_blocks(k_batch_stage<KK, false, STAGE>, SW_COLS * SW_WAVES);
    });
}

static int blocks_step(int K, bool tracked)
{
    return with_k_bstrip(K, [&]<int KK>() {
        return tracked ? resident_blocks(k_batch_step<KK, true>, SW_COLS * SW_WAVES)
                       : resident_blocks(k_batch_step<KK, false>, SW_COLS * SW_WAVES);
    });
}

template <int MODE>
static int blocks_x()
{
    return resident_blocks(k_batch_x<MODE>, 256);
}

template <int MODE>
static int blocks_col(int K, int shape, bool mixed)
{
    if (mixed)
        return with_k_mixed(K, [&]<int KK, class S>() { return resident_blocks(k_batch_col<KK, MODE, S, FORM_MIXED>, S::NTC); });
    return with_k_shape(K, shape, [&]<int KK, class S>() { return resident_blocks(k_batch_col<KK, MODE, S, FORM_FP64>, S::NTC); });
}

// The Pade line of a member as the planner sees it (no table pointers).
static PadeLine host_line(int n_in)
{
    PadeLine L{};
    L.n_in = n_in;
    L.n_out = n_in - 1;
    L.all = L.n_out <= 2 * PADE_B;
    L.b = L.all ? L.n_out : PADE_B;
    return L;
}

// Plan of one strip solve of a member for `slots` of the resident wave
// slots (its share of the batch), and the estimated cost of each item.
template <int MODE>
static bool member_plan(int K, const UGrid& g, const PadeLine& L, int slots, StripPlan& plan, std::vector<double>* cost)
{
    return with_k_bstrip(K, [&]<int KK>() {
        using SS = StripShape<KK, MODE, BS_U, BS_LA>;
        if (!strip_plan<SS, KK, BS_U>(g, L, slots, std::max(1, slots / 3), plan)) return false;
        if (cost) {
            cost->resize(plan.items());
            for (int it = 0; it < plan.items(); ++it) {
                int strip, y0, tr;
                bool up;
                plan.item(it, strip, y0, tr, up);
                const int v = strip_variant<SS, KK>(g, L, g.lo[0] + strip * SS::OW, y0, tr);
                (*cost)[it] = STRIP_COST[v] * (tr + STRIP_FILL_STEPS);
            }
        }
        return true;
    });
}

}  // namespace c4m

using namespace c4m;

// Internal hooks of the single-problem runtime (c4m_host.hip).
namespace c4m {
c4m_status problem_view(c4m_problem* p, ProblemView* v);
c4m_status problem_prepare(c4m_problem* p);     // carried-Laplacian conversion before stepping
const std::vector<Launch3>* problem_step3_plan(c4m_problem* p);
c4m_status problem_create_owned(const c4m_config* cfg, void* ws, size_t bytes, hipStream_t st,
                                c4m_problem** out);
void problem_add_steps(c4m_problem* p, int64_t n);
void problem_destroy_owned(c4m_problem* p);
const c4m_config* problem_config(const c4m_problem* p);
c4m_status set_error(c4m_status s, const char* msg);
}  // namespace c4m

struct c4m_batch {
    int count = 0;
    c4m_config base{};
    hipStream_t stream = nullptr;
    std::vector<c4m_problem*> probs;
    BatchProb* d_probs = nullptr;
    Item* d_items = nullptr;
    int* d_ctr = nullptr;          // [NSTMAX][16] chunk counters, finished, err, done[count][NSTMAX]
    Sched sched{};
    int nst = 0;                   // stages (launches of the column-tile form)
    int total[NSTMAX] = {};
    Coef coef{};
    PadeTaps taps_xe{}, taps_xh{};
    ChebSchedule cheb{};
    int blocks[NSTMAX] = {};       // workgroups of each launch
    bool owns = true;              // problems created by (and destroyed with) the batch
    bool strips = false;           // strip form: one launch per step
    // 3D members: every launch of the recorded step over all members
    bool three_d = false;
    struct L3 {
        Launch3 proto;             // member 0's record (kind, template choice, class)
        size_t off;                // its member arguments in the table
        unsigned blocks;           // workgroups over all members
    };
    std::vector<L3> l3;
    char* d_tab3 = nullptr;
    PadeTaps taps3[2]{};
    std::map<int64_t, std::pair<hipGraph_t, hipGraphExec_t>> graphs;   // captured runs of steps
    // C4M_FLAG_PROFILE: every launch bracketed by HIP events on the stream
    // (no graph, no host wait); read and summed by c4m_batch_get_info
    struct Rec {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double kernel_ms[C4M_K_COUNT] = {};
    int64_t kernel_launches[C4M_K_COUNT] = {};
    double alg_bytes[C4M_K_COUNT] = {};
};

namespace {

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

constexpr int CTR_STAGE = 16;      // ints per stage's chunk counters (one 64-byte line)
constexpr int DEFAULT_WAIT_LIMIT = 1 << 24;
constexpr int GRAPH_STEPS = 32;    // launches per captured graph

c4m_status check_uniform(const c4m_config* cfgs, int32_t count)
{
    if (!cfgs || count < 1) return set_error(C4M_EINVAL, "empty batch");
    for (int i = 0; i < count; ++i) {
        const c4m_config& c = cfgs[i];
        if (c.dim != cfgs[0].dim) return set_error(C4M_EINVAL, "batched problems must share the dimension");
        if (c.dim == 3 && (c.precision != C4M_FP64 || c.solver != C4M_SOLVER_CHEBYSHEV))
            return set_error(C4M_EINVAL, "batched 3D problems: FP64 Chebyshev form only");
        if (c.scheme != C4M_SCHEME_C4) return set_error(C4M_EINVAL, "batched form runs the compact scheme");
        if (c.solver != C4M_SOLVER_CHEBYSHEV)
            return set_error(C4M_EINVAL, "batched form runs the fused Chebyshev solve only");
        if (c.cfl != cfgs[0].cfl || c.z != cfgs[0].z || c.closure != cfgs[0].closure ||
            c.lap_mode != cfgs[0].lap_mode || c.precision != cfgs[0].precision ||
            c.solver != cfgs[0].solver || c.sweeps != cfgs[0].sweeps || c.tile_x != cfgs[0].tile_x ||
            c.tile_y != cfgs[0].tile_y || c.batch_wait_limit != cfgs[0].batch_wait_limit)
            return set_error(C4M_EINVAL, "batched problems must share cfl, z, closure, lap_mode, precision, solver");
        if (c.batch_wait_limit < 0) return set_error(C4M_EINVAL, "batch_wait_limit must be >= 0");
        size_t b = 0;
        c4m_status s = c4m_workspace_bytes(&c, &b);
        if (s != C4M_OK) return s;
    }
    return C4M_OK;
}

// Chebyshev applications per solve of a configuration (as c4m_create sets them)
int config_sweeps(const c4m_config& c)
{
    const double r = c.cfl, alpha = 1.0 + 2.0 / (r * r), beta = r * r / 24.0;
    if (c.precision == C4M_FP32_REFINED) return 2 * (c.sweeps > 0 ? c.sweeps : 2) + 1;
    if (c.sweeps > 0) return c.sweeps;
    const double lmin = alpha, lmax = alpha + 16.0 / 3.0 * beta;
    const double sigma = (lmax + lmin) / (lmax - lmin);
    int k = 1;
    while (k < MAX_SWEEPS && 1.0 / cosh((k + 1) * acosh(sigma)) > CHEB_TOL) ++k;
    return k;
}

// Work of the batch: member descriptors, stage item tables, launch sizes.
struct Layout {
    std::vector<BatchProb> probs;
    std::vector<Item> items[NSTMAX];
    int nst = 0;
    bool strips = false;
    int blocks[NSTMAX] = {};
};

// Everything except the member pointers (filled by build_tables) is a
// function of the configurations, so the table size is known before any
// problem exists.
c4m_status plan_layout(const c4m_config* cfgs, int count, bool strips_ok, Layout& lay)
{
    const c4m_config& c0 = cfgs[0];
    const bool mixed = c0.precision == C4M_FP32_REFINED;
    const bool tracked = c0.lap_mode == C4M_LAP_TRACKED;
    const int shape = c0.tile_x;
    const int K = config_sweeps(c0);
    lay.strips = strips_ok && strip_form_2d(shape, mixed, K);
    lay.nst = lay.strips ? 4 : 5;
    lay.probs.assign(count, BatchProb{});
    std::vector<std::vector<double>> ccost[2];     // strip form: item costs of CE and CH per member
    for (int k = 0; k < 2; ++k) ccost[k].resize(count);
    int step_blocks = 0;
    double cells_total = 0.0;
    for (int i = 0; i < count; ++i) cells_total += (double)cfgs[i].n * cfgs[i].n;
    if (lay.strips) step_blocks = blocks_step(K, tracked);
    const int slots_total = step_blocks * SW_WAVES;
    for (int i = 0; i < count; ++i) {
        const int N = cfgs[i].n;
        BatchProb& d = lay.probs[i];
        const PadeLine l1 = host_line(N), l0 = host_line(N + 1);   // Step 1 y-lines (half), Step 2 (node)
        d.xe_tx = xe_tiles_x(l1.n_out);
        d.xh_tx = xlines_tiles_x(l0.n_out);
        if (lay.strips) {
            d.xe_tiles = d.xe_tx * xe_tiles_y(N);
            d.xh_tiles = d.xh_tx * xlines_tiles_y(N);
            const int nbx = (N + 1 + 255) / 256;
            d.items[ST_XE] = d.xe_tiles + nbx * band_rows(l1) * 2;
            d.items[ST_XH] = d.xh_tiles + nbx * band_rows(l0) * 2;
            // the member's share of the resident wave slots: long segments
            // (little halo and window refill), enough of them to balance
            const int slots = std::max(8, (int)(slots_total * ((double)N * N / cells_total)));
            std::vector<double> chx_cost, chy_cost;
            bool ok = tracked ? member_plan<COL_E_TRACKED>(K, ugrid_ez(N), l1, slots, d.plan[0], &ccost[0][i])
                              : member_plan<COL_E_DISCRETE>(K, ugrid_ez(N), l1, slots, d.plan[0], &ccost[0][i]);
            ok = ok && (tracked ? member_plan<COL_HX_TRACKED>(K, ugrid_hx(N), l0, slots, d.plan[1], &chx_cost)
                                : member_plan<COL_HX_DISCRETE>(K, ugrid_hx(N), l0, slots, d.plan[1], &chx_cost));
            ok = ok && member_plan<COL_HY>(K, ugrid_hy(N), l0, slots, d.plan[2], &chy_cost);
            if (!ok) return set_error(C4M_EINVAL, "no strip plan for a batch member");
            d.items[ST_CE] = d.plan[0].items();
            d.n_chx = d.plan[1].items();
            d.items[ST_CH] = d.n_chx + d.plan[2].items();
            ccost[1][i] = chx_cost;
            ccost[1][i].insert(ccost[1][i].end(), chy_cost.begin(), chy_cost.end());
        } else {
            d.xe_tiles = d.xe_tx * xe_tiles_y(N);
            d.xh_tiles = d.xh_tx * xlines_tiles_y(N);
            d.items[ST_XE] = d.xe_tiles;
            d.items[ST_XH] = d.xh_tiles;
            d.items[ST_CE] = col_tiles_k(K, shape, mixed, ugrid_ez(N), &d.ce_ty);
            d.items[ST_CH] = col_tiles_k(K, shape, mixed, ugrid_hx(N), &d.chx_ty);
            d.items[ST_CHY] = col_tiles_k(K, shape, mixed, ugrid_hy(N), &d.chy_ty);
        }
    }
    // x-line stages: problem by problem, the largest first (their solves are
    // the longest, and they wait for these), tiles of a problem together so
    // the tiles one XCD runs at a time share their halo rows in its L2
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cfgs[a].n > cfgs[b].n; });
    for (int st : {ST_XE, ST_XH})
        for (int i : order)
            for (int l = 0; l < lay.probs[i].items[st]; ++l) lay.items[st].push_back(Item{i, l});
    if (lay.strips) {
        // solve stages: longest items first over all problems (runs of four
        // similar items per workgroup), laid out so that every XCD chunk of
        // the table holds a similar mix
        for (int k = 0; k < 2; ++k) {
            const int st = k == 0 ? ST_CE : ST_CH;
            // cost bins of about 15 %, longest first; inside a bin the
            // items of one problem, by segment, then strip, so the four
            // waves of a workgroup walk neighbouring strips of one segment
            // and share their halo columns in L1/L2
            struct C {
                int bin, seg, strip;
                Item it;
            };
            std::vector<C> all;
            for (int i = 0; i < count; ++i)
                for (int l = 0; l < (int)ccost[k][i].size(); ++l) {
                    const BatchProb& d = lay.probs[i];
                    const int hy = k == 1 && l >= d.n_chx;           // Step 2: Hy strips after the Hx strips
                    const StripPlan& pl = k == 0 ? d.plan[0] : d.plan[hy ? 2 : 1];
                    int strip, y0, tr;
                    bool up;
                    pl.item(hy ? l - d.n_chx : l, strip, y0, tr, up);
                    const int bin = (int)floor(log(std::max(ccost[k][i][l], 1.0)) / log(1.15));
                    all.push_back(C{bin, y0 + hy * 65536, strip, Item{i, l}});
                }
            std::stable_sort(all.begin(), all.end(), [](const C& a, const C& b) {
                if (a.bin != b.bin) return a.bin > b.bin;
                if (a.it.p != b.it.p) return a.it.p < b.it.p;
                if (a.seg != b.seg) return a.seg < b.seg;
                return a.strip < b.strip;
            });
            const int total = (int)all.size();
            const int per = (total + NXCD - 1) / NXCD;
            std::vector<Item>& out = lay.items[st];
            out.assign(total, Item{0, 0});
            // deal runs of SW_WAVES items to the chunks in turn
            std::vector<int> fill(NXCD, 0);
            int c = 0;
            for (int j = 0; j < total;) {
                for (int tries = 0; tries < NXCD; ++tries, c = (c + 1) % NXCD)
                    if (fill[c] < std::min(per, total - c * per)) break;
                const int room = std::min(per, total - c * per) - fill[c];
                const int run = std::min({SW_WAVES, room, total - j});
                for (int r = 0; r < run; ++r) out[c * per + fill[c] + r] = all[j + r].it;
                fill[c] += run;
                j += run;
                c = (c + 1) % NXCD;
            }
        }
        if (c0.tile_y != 1) {
            // one launch per stage (the default: faster than the single
            // launch, whose cross-XCD fences cost more than the launch
            // boundaries)
            lay.blocks[ST_XE] = blocks_stage<ST_XE>(K, tracked);
            lay.blocks[ST_CE] = blocks_stage<ST_CE>(K, tracked);
            lay.blocks[ST_XH] = blocks_stage<ST_XH>(K, tracked);
            lay.blocks[ST_CH] = blocks_stage<ST_CH>(K, tracked);
        } else {
            lay.blocks[0] = step_blocks;
        }
    } else {
        for (int st : {ST_CE, ST_CH, ST_CHY})
            for (int i = 0; i < count; ++i)
                for (int l = 0; l < lay.probs[i].items[st]; ++l) lay.items[st].push_back(Item{i, l});
        const int mult = c0.tile_y > 0 ? c0.tile_y : 1;   // persistent grid multiplier
        lay.blocks[ST_XE] = (tracked ? blocks_x<XL_E_TRACKED>() : blocks_x<XL_E_DISCRETE>()) * mult;
        lay.blocks[ST_XH] = (tracked ? blocks_x<XL_H_TRACKED>() : blocks_x<XL_H_DISCRETE>()) * mult;
        lay.blocks[ST_CE] = (tracked ? blocks_col<COL_E_TRACKED>(K, shape, mixed) : blocks_col<COL_E_DISCRETE>(K, shape, mixed)) * mult;
        lay.blocks[ST_CH] = (tracked ? blocks_col<COL_HX_TRACKED>(K, shape, mixed) : blocks_col<COL_HX_DISCRETE>(K, shape, mixed)) * mult;
        lay.blocks[ST_CHY] = blocks_col<COL_HY>(K, shape, mixed) * mult;
    }
    return C4M_OK;
}

size_t layout_bytes(const Layout& lay, int count)
{
    size_t items = 0;
    for (int st = 0; st < NSTMAX; ++st) items += lay.items[st].size();
    return a256(sizeof(BatchProb) * count) + a256(sizeof(Item) * items) +
           a256(sizeof(int) * ((NSTMAX + 2) * CTR_STAGE + (size_t)count * NSTMAX));
}

// the strip form needs every member's used workspace below one buffer
// resource's range
bool strips_fit(c4m_problem* const* probs, int count)
{
    for (int i = 0; i < count; ++i) {
        ProblemView v{};
        problem_view(probs[i], &v);
        if (!v.yband || v.used >= (size_t)0xFFFFF000u) return false;
    }
    return true;
}

bool strips_fit_cfg(const c4m_config* cfgs, int count)
{
    for (int i = 0; i < count; ++i) {
        size_t b = 0;
        if (c4m_workspace_bytes(&cfgs[i], &b) != C4M_OK || b >= (size_t)0xFFFFF000u) return false;
    }
    return true;
}

// kernel class of each stage launch
int stage_class(int st)
{
    return st == ST_XE ? C4M_K_RHS_E : (st == ST_CE ? C4M_K_SOLVE_E : (st == ST_XH ? C4M_K_RHS_H : C4M_K_SOLVE_H));
}

hipEvent_t pool_event(c4m_batch* b)
{
    if (!b->pool.empty()) {
        hipEvent_t e = b->pool.back();
        b->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

c4m_status flush_batch_profile(c4m_batch* b)
{
    if (b->pending.empty()) return C4M_OK;
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return set_error(C4M_EDEVICE, hipGetErrorString(e));
    for (auto& r : b->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            b->kernel_ms[r.cls] += ms;
            b->kernel_launches[r.cls] += 1;
        }
        b->pool.push_back(r.a);
        b->pool.push_back(r.b);
    }
    b->pending.clear();
    return C4M_OK;
}

// record the event before (open) or after (close) a launch of class cls
c4m_status mark(c4m_batch* b, int cls, bool open)
{
    if (!(b->base.flags & C4M_FLAG_PROFILE)) return C4M_OK;
    if (open) {
        if (b->pending.size() >= 2048) {
            c4m_status s = flush_batch_profile(b);
            if (s != C4M_OK) return s;
        }
        hipEvent_t a = pool_event(b), z = pool_event(b);
        if (!a || !z) return set_error(C4M_EDEVICE, "hipEventCreate");
        b->pending.push_back({cls, a, z});
        return hipEventRecord(a, b->stream) == hipSuccess ? C4M_OK : set_error(C4M_EDEVICE, "hipEventRecord");
    }
    return hipEventRecord(b->pending.back().b, b->stream) == hipSuccess ? C4M_OK
                                                                         : set_error(C4M_EDEVICE, "hipEventRecord");
}

c4m_status launch_step(c4m_batch* b)
{
    const bool tracked = b->base.lap_mode == C4M_LAP_TRACKED;
    const bool mixed = b->base.precision == C4M_FP32_REFINED;
    const int K = b->cheb.sweeps;
    const BatchProb* bp = b->d_probs;
    hipError_t e = hipSuccess;
    if (b->strips && b->base.tile_y != 1) {
        for (int st = 0; st < 4 && e == hipSuccess; ++st) {
            const int g = std::max(1, std::min(b->blocks[st], b->total[st]));
            if (mark(b, stage_class(st), true) != C4M_OK) return C4M_EDEVICE;
            if (st == ST_XH && b->total[st] > 0) {
                // Step 2 x-lines as a plain grid (measured faster than the
                // persistent claim: 784 against 910 us on the 512-cavity mix;
                // the Step 1 tiles, four workgroups per CU by LDS, are
                // faster persistent: 1173 against 1273 us)
                const dim3 gx((unsigned)(NXCD * ((b->total[st] + NXCD - 1) / NXCD)));
                if (tracked)
                    hipLaunchKernelGGL((k_batch_xstage<true, ST_XH>), gx, dim3(SW_COLS * SW_WAVES), 0, b->stream, bp,
                                       b->sched, b->coef, b->taps_xh);
                else
                    hipLaunchKernelGGL((k_batch_xstage<false, ST_XH>), gx, dim3(SW_COLS * SW_WAVES), 0, b->stream, bp,
                                       b->sched, b->coef, b->taps_xh);
                e = hipGetLastError();
                if (e == hipSuccess && mark(b, stage_class(st), false) != C4M_OK) return C4M_EDEVICE;
                continue;
            }
            e = with_k_bstrip(K, [&]<int KK>() {
                auto go = [&]<int ST>() {
                    if (tracked)
                        hipLaunchKernelGGL((k_batch_stage<KK, true, ST>), dim3(g), dim3(SW_COLS * SW_WAVES), 0,
                                           b->stream, bp, b->sched, b->coef, b->taps_xh, b->cheb);
                    else
                        hipLaunchKernelGGL((k_batch_stage<KK, false, ST>), dim3(g), dim3(SW_COLS * SW_WAVES), 0,
                                           b->stream, bp, b->sched, b->coef, b->taps_xh, b->cheb);
                };
                if (st == ST_XE) go.template operator()<ST_XE>();
                else if (st == ST_CE) go.template operator()<ST_CE>();
                else if (st == ST_XH) go.template operator()<ST_XH>();
                else go.template operator()<ST_CH>();
                return hipGetLastError();
            });
            if (e == hipSuccess && mark(b, stage_class(st), false) != C4M_OK) return C4M_EDEVICE;
        }
        return e == hipSuccess ? C4M_OK : set_error(C4M_EDEVICE, hipGetErrorString(e));
    }
    if (b->strips) {
        const int g = std::max(1, b->blocks[0]);
        if (mark(b, C4M_K_STEP, true) != C4M_OK) return C4M_EDEVICE;
        e = with_k_bstrip(K, [&]<int KK>() {
            if (tracked)
                hipLaunchKernelGGL((k_batch_step<KK, true>), dim3(g), dim3(SW_COLS * SW_WAVES), 0, b->stream, bp,
                                   b->sched, b->coef, b->taps_xh, b->cheb);
            else
                hipLaunchKernelGGL((k_batch_step<KK, false>), dim3(g), dim3(SW_COLS * SW_WAVES), 0, b->stream, bp,
                                   b->sched, b->coef, b->taps_xh, b->cheb);
            return hipGetLastError();
        });
        if (e == hipSuccess && mark(b, C4M_K_STEP, false) != C4M_OK) return C4M_EDEVICE;
        return e == hipSuccess ? C4M_OK : set_error(C4M_EDEVICE, hipGetErrorString(e));
    }
    const int shape = b->base.tile_x;
    for (int st = 0; st < b->nst && e == hipSuccess; ++st) {
        if (!b->total[st]) continue;
        const int g = std::max(1, std::min(b->blocks[st], b->total[st]));
        const Sched& sc = b->sched;
        const int cls = st == ST_CHY ? C4M_K_SOLVE_H : stage_class(st);
        if (mark(b, cls, true) != C4M_OK) return C4M_EDEVICE;
        if (st == ST_XE || st == ST_XH) {
            const PadeTaps& taps = st == ST_XE ? b->taps_xe : b->taps_xh;
            if (st == ST_XE && tracked)
                hipLaunchKernelGGL(k_batch_x<XL_E_TRACKED>, dim3(g), dim3(256), 0, b->stream, bp, sc, st, b->coef, taps);
            else if (st == ST_XE)
                hipLaunchKernelGGL(k_batch_x<XL_E_DISCRETE>, dim3(g), dim3(256), 0, b->stream, bp, sc, st, b->coef, taps);
            else if (tracked)
                hipLaunchKernelGGL(k_batch_x<XL_H_TRACKED>, dim3(g), dim3(256), 0, b->stream, bp, sc, st, b->coef, taps);
            else
                hipLaunchKernelGGL(k_batch_x<XL_H_DISCRETE>, dim3(g), dim3(256), 0, b->stream, bp, sc, st, b->coef, taps);
            e = hipGetLastError();
            if (e == hipSuccess && mark(b, cls, false) != C4M_OK) return C4M_EDEVICE;
            continue;
        }
        const int mode = st == ST_CE ? (tracked ? COL_E_TRACKED : COL_E_DISCRETE)
                                     : (st == ST_CH ? (tracked ? COL_HX_TRACKED : COL_HX_DISCRETE) : COL_HY);
        const PadeTaps& taps = st == ST_CE ? b->taps_xe : b->taps_xh;
        auto launch = [&]<int MODE>() {
            if (mixed)
                return with_k_mixed(K, [&]<int KK, class S>() {
                    hipLaunchKernelGGL((k_batch_col<KK, MODE, S, FORM_MIXED>), dim3(g), dim3(S::NTC), 0, b->stream,
                                       bp, sc, st, b->coef, taps, b->cheb);
                    return hipGetLastError();
                });
            return with_k_shape(K, shape, [&]<int KK, class S>() {
                hipLaunchKernelGGL((k_batch_col<KK, MODE, S, FORM_FP64>), dim3(g), dim3(S::NTC), 0, b->stream, bp,
                                   sc, st, b->coef, taps, b->cheb);
                return hipGetLastError();
            });
        };
        switch (mode) {
            case COL_E_TRACKED: e = launch.template operator()<COL_E_TRACKED>(); break;
            case COL_E_DISCRETE: e = launch.template operator()<COL_E_DISCRETE>(); break;
            case COL_HX_TRACKED: e = launch.template operator()<COL_HX_TRACKED>(); break;
            case COL_HX_DISCRETE: e = launch.template operator()<COL_HX_DISCRETE>(); break;
            default: e = launch.template operator()<COL_HY>(); break;
        }
        if (e == hipSuccess && mark(b, cls, false) != C4M_OK) return C4M_EDEVICE;
    }
    return e == hipSuccess ? C4M_OK : set_error(C4M_EDEVICE, hipGetErrorString(e));
}

std::vector<c4m_config> member_configs(c4m_problem* const* probs, int count)
{
    std::vector<c4m_config> cfgs(count);
    for (int i = 0; i < count; ++i) cfgs[i] = *problem_config(probs[i]);
    return cfgs;
}

// Fill the member pointers of the layout from the problems and upload the
// tables at `cur` (`bytes` available).
c4m_status build_tables(c4m_batch* b, Layout& lay, char* cur, size_t bytes)
{
    const int count = b->count;
    if (bytes < layout_bytes(lay, count)) return set_error(C4M_ENOMEM, "table space smaller than needed");
    b->d_probs = (BatchProb*)cur;
    cur += a256(sizeof(BatchProb) * count);
    b->d_items = (Item*)cur;
    size_t nitems = 0;
    for (int st = 0; st < NSTMAX; ++st) nitems += lay.items[st].size();
    cur += a256(sizeof(Item) * nitems);
    b->d_ctr = (int*)cur;
    b->strips = lay.strips;
    b->nst = lay.nst;
    const bool tracked = b->base.lap_mode == C4M_LAP_TRACKED;
    for (int i = 0; i < count; ++i) {
        ProblemView v{};
        problem_view(b->probs[i], &v);
        const int N = v.N;
        BatchProb& d = lay.probs[i];
        d.xe = XArgs{v.f[C4M_HY], v.tmp[0], v.tmp[1], N, v.P, v.line[1]};
        d.xh = XArgs{tracked ? v.ge[2] : v.f[C4M_EZ], v.tmp[0], v.tmp[1], N, v.P, v.line[0]};
        d.ce = ColArgs{v.f[C4M_HX], v.tmp[0], v.tmp[1], v.f[C4M_EZ], v.ge[2], ugrid_ez(N), N, v.P};
        d.chx = ColArgs{tracked ? v.ge[2] : v.f[C4M_EZ], nullptr, nullptr, v.f[C4M_HX], nullptr, ugrid_hx(N), N, v.P};
        d.chy = ColArgs{nullptr, v.tmp[1], nullptr, v.f[C4M_HY], nullptr, ugrid_hy(N), N, v.P};
        if (b->strips) d.ce.yb = d.chx.yb = d.chy.yb = v.yband;
        if (i == 0) {
            b->coef = v.coef;
            b->taps_xe = v.taps[1];
            b->taps_xh = v.taps[0];
            b->cheb = v.cheb;
        }
    }
    if (b->cheb.sweeps != config_sweeps(b->base))
        return set_error(C4M_EINVAL, "batch plan and members disagree on the Chebyshev sweep count");
    std::vector<Item> flat;
    size_t off[NSTMAX];
    for (int st = 0; st < NSTMAX; ++st) {
        off[st] = flat.size();
        flat.insert(flat.end(), lay.items[st].begin(), lay.items[st].end());
        b->total[st] = (int)lay.items[st].size();
        b->blocks[st] = lay.blocks[st];
    }
    Sched& sc = b->sched;
    for (int st = 0; st < NSTMAX; ++st)
        sc.st[st] = Stage{b->d_items + off[st], b->total[st], b->d_ctr + st * CTR_STAGE};
    sc.finished = b->d_ctr + NSTMAX * CTR_STAGE;
    sc.err = b->d_ctr + (NSTMAX + 1) * CTR_STAGE;
    sc.done = b->d_ctr + (NSTMAX + 2) * CTR_STAGE;
    sc.count = count;
    sc.wait_limit = b->base.batch_wait_limit > 0 ? b->base.batch_wait_limit : DEFAULT_WAIT_LIMIT;
    const size_t ctr_bytes = sizeof(int) * ((NSTMAX + 2) * CTR_STAGE + (size_t)count * NSTMAX);
    hipError_t e = hipMemcpyAsync(b->d_probs, lay.probs.data(), sizeof(BatchProb) * count, hipMemcpyHostToDevice,
                                  b->stream);
    if (e == hipSuccess && !flat.empty())
        e = hipMemcpyAsync(b->d_items, flat.data(), sizeof(Item) * flat.size(), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_ctr, 0, ctr_bytes, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    return e == hipSuccess ? C4M_OK : set_error(C4M_EDEVICE, hipGetErrorString(e));
}

}  // namespace

namespace c4m {

// Table bytes of the batched 3D step: every launch's member arguments.
c4m_status plan_batch3(c4m_problem* const* probs, int count, std::vector<c4m_batch::L3>* l3, size_t* bytes)
{
    const std::vector<Launch3>* p0 = problem_step3_plan(probs[0]);
    if (!p0) return set_error(C4M_EINVAL, "3D batch members must take the FP64 Chebyshev form");
    size_t off = 0;
    for (size_t i = 0; i < p0->size(); ++i) {
        unsigned blocks = 0;
        for (int m = 0; m < count; ++m) {
            const std::vector<Launch3>* pm = problem_step3_plan(probs[m]);
            if (!pm || pm->size() != p0->size() || (*pm)[i].kind != (*p0)[i].kind || (*pm)[i].axis != (*p0)[i].axis ||
                (*pm)[i].mode != (*p0)[i].mode || (*pm)[i].first != (*p0)[i].first || (*pm)[i].out != (*p0)[i].out)
                return set_error(C4M_EINVAL, "3D batch members differ in their step");
            blocks += (*pm)[i].gx * (*pm)[i].gy * (*pm)[i].gz;
        }
        if (l3) l3->push_back(c4m_batch::L3{(*p0)[i], off, blocks});
        off = (off + (size_t)count * launch3_arg_bytes((*p0)[i]) + 255) / 256 * 256;
    }
    *bytes = off + 256;
    return C4M_OK;
}

c4m_status build_batch3(c4m_batch* b, char* d_tab, size_t bytes)
{
    size_t need = 0;
    b->l3.clear();
    c4m_status s = plan_batch3(b->probs.data(), b->count, &b->l3, &need);
    if (s != C4M_OK) return s;
    if (bytes < need) return set_error(C4M_ENOMEM, "table space smaller than c4m_batch_tables_bytes");
    std::vector<char> host(need, 0);
    for (size_t i = 0; i < b->l3.size(); ++i) {
        const size_t ab = launch3_arg_bytes(b->l3[i].proto);
        int first = 0;
        for (int m = 0; m < b->count; ++m) {
            const Launch3& r = (*problem_step3_plan(b->probs[m]))[i];
            launch3_pack(r, first, host.data() + b->l3[i].off + (size_t)m * ab);
            first += (int)(r.gx * r.gy * r.gz);
        }
    }
    b->d_tab3 = d_tab;
    hipError_t e = hipMemcpyAsync(d_tab, host.data(), need, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return set_error(C4M_EDEVICE, "3D batch table upload");
    ProblemView v{};
    problem_view(b->probs[0], &v);
    b->taps3[0] = v.taps[0];
    b->taps3[1] = v.taps[1];
    b->three_d = true;
    return C4M_OK;
}

c4m_status launch_step3b(c4m_batch* b)
{
    const size_t n = b->l3.size();
    for (size_t i = 0; i < n;) {
        size_t j = i;
        while (j < n && b->l3[j].proto.cls == b->l3[i].proto.cls && b->l3[j].proto.group == b->l3[i].proto.group) ++j;
        if (mark(b, b->l3[i].proto.cls, true) != C4M_OK) return C4M_EDEVICE;
        for (size_t k = i; k < j; ++k) {
            const c4m_batch::L3& l = b->l3[k];
            hipError_t e = launch3_batched(b->stream, l.proto, b->d_tab3 + l.off, b->count, l.blocks, b->taps3);
            if (e != hipSuccess) return set_error(C4M_EDEVICE, hipGetErrorString(e));
        }
        if (mark(b, b->l3[i].proto.cls, false) != C4M_OK) return C4M_EDEVICE;
        i = j;
    }
    return C4M_OK;
}

}  // namespace c4m

extern "C" {

c4m_status c4m_batch_workspace_bytes(const c4m_config* cfgs, int32_t count, size_t* bytes)
{
    c4m_status s = check_uniform(cfgs, count);
    if (s != C4M_OK) return s;
    if (!bytes) return set_error(C4M_EINVAL, "null bytes");
    if (cfgs[0].dim == 3) return set_error(C4M_EINVAL, "3D batches are formed from existing problems (c4m_batch_create_from)");
    Layout lay;
    s = plan_layout(cfgs, count, strips_fit_cfg(cfgs, count), lay);
    if (s != C4M_OK) return s;
    size_t tot = layout_bytes(lay, count);
    for (int i = 0; i < count; ++i) {
        size_t b = 0;
        c4m_workspace_bytes(&cfgs[i], &b);
        tot += a256(b);
    }
    *bytes = tot;
    return C4M_OK;
}

c4m_status c4m_batch_create(const c4m_config* cfgs, int32_t count, void* d_workspace, size_t bytes,
                            void* hip_stream, c4m_batch** out)
{
    if (!out) return set_error(C4M_EINVAL, "null out");
    *out = nullptr;
    size_t need = 0;
    c4m_status s = c4m_batch_workspace_bytes(cfgs, count, &need);
    if (s != C4M_OK) return s;
    if (!d_workspace || ((uintptr_t)d_workspace & 255)) return set_error(C4M_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < need) return set_error(C4M_ENOMEM, "workspace smaller than c4m_batch_workspace_bytes");
    Layout lay;
    s = plan_layout(cfgs, count, strips_fit_cfg(cfgs, count), lay);
    if (s != C4M_OK) return s;
    c4m_batch* b = new (std::nothrow) c4m_batch();
    if (!b) return set_error(C4M_ENOMEM, "host allocation");
    b->count = count;
    b->base = cfgs[0];
    b->stream = (hipStream_t)hip_stream;
    char* tables = (char*)d_workspace;
    const size_t tb = layout_bytes(lay, count);
    char* cur = tables + tb;
    for (int i = 0; i < count && s == C4M_OK; ++i) {
        size_t pb = 0;
        c4m_workspace_bytes(&cfgs[i], &pb);
        c4m_problem* p = nullptr;
        s = problem_create_owned(&cfgs[i], cur, pb, b->stream, &p);
        if (s != C4M_OK) break;
        cur += a256(pb);
        b->probs.push_back(p);
    }
    if (s == C4M_OK) s = build_tables(b, lay, tables, tb);
    if (s != C4M_OK) {
        for (auto* p : b->probs) problem_destroy_owned(p);
        delete b;
        return s;
    }
    *out = b;
    return C4M_OK;
}

c4m_status c4m_batch_tables_bytes(c4m_problem* const* probs, int32_t count, size_t* bytes)
{
    if (!probs || count < 1 || !bytes) return set_error(C4M_EINVAL, "bad arguments");
    for (int i = 0; i < count; ++i)
        if (!probs[i]) return set_error(C4M_EINVAL, "null problem");
    std::vector<c4m_config> cfgs = member_configs(probs, count);
    c4m_status s = check_uniform(cfgs.data(), count);
    if (s != C4M_OK) return s;
    if (cfgs[0].dim == 3) return plan_batch3(probs, count, nullptr, bytes);
    Layout lay;
    s = plan_layout(cfgs.data(), count, strips_fit(probs, count), lay);
    if (s != C4M_OK) return s;
    *bytes = layout_bytes(lay, count);
    return C4M_OK;
}

c4m_status c4m_batch_create_from(c4m_problem* const* probs, int32_t count, void* d_tables, size_t bytes,
                                 void* hip_stream, c4m_batch** out)
{
    if (!out || !probs || count < 1) return set_error(C4M_EINVAL, "bad arguments");
    *out = nullptr;
    if (!d_tables || ((uintptr_t)d_tables & 255)) return set_error(C4M_EINVAL, "tables must be 256-byte aligned");
    for (int i = 0; i < count; ++i)
        if (!probs[i]) return set_error(C4M_EINVAL, "null problem");
    std::vector<c4m_config> cfgs = member_configs(probs, count);
    c4m_status s = check_uniform(cfgs.data(), count);
    if (s != C4M_OK) return s;
    if (cfgs[0].dim == 3) {
        c4m_batch* b = new (std::nothrow) c4m_batch();
        if (!b) return set_error(C4M_ENOMEM, "host allocation");
        b->count = count;
        b->base = cfgs[0];
        b->stream = (hipStream_t)hip_stream;
        b->owns = false;
        b->probs.assign(probs, probs + count);
        s = build_batch3(b, (char*)d_tables, bytes);
        if (s != C4M_OK) {
            delete b;
            return s;
        }
        *out = b;
        return C4M_OK;
    }
    Layout lay;
    s = plan_layout(cfgs.data(), count, strips_fit(probs, count), lay);
    if (s != C4M_OK) return s;
    if (bytes < layout_bytes(lay, count)) return set_error(C4M_ENOMEM, "table space smaller than c4m_batch_tables_bytes");
    c4m_batch* b = new (std::nothrow) c4m_batch();
    if (!b) return set_error(C4M_ENOMEM, "host allocation");
    b->count = count;
    b->base = cfgs[0];
    b->stream = (hipStream_t)hip_stream;
    b->owns = false;
    b->probs.assign(probs, probs + count);
    s = build_tables(b, lay, (char*)d_tables, bytes);
    if (s != C4M_OK) {
        delete b;
        return s;
    }
    *out = b;
    return C4M_OK;
}

c4m_status c4m_batch_problem(c4m_batch* b, int32_t i, c4m_problem** out)
{
    if (!b || !out || i < 0 || i >= b->count) return set_error(C4M_EINVAL, "bad batch index");
    *out = b->probs[i];
    return C4M_OK;
}

c4m_status c4m_batch_step(c4m_batch* b, int64_t nsteps)
{
    if (!b || nsteps < 0) return set_error(C4M_EINVAL, "bad step count");
    if (nsteps == 0) return C4M_OK;
    for (auto* p : b->probs) {
        c4m_status s = problem_prepare(p);
        if (s != C4M_OK) return s;
    }
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    bool direct = (b->base.flags & (C4M_FLAG_PROFILE | C4M_FLAG_DIRECT)) || !b->stream;
    if (!direct && hipStreamIsCapturing(b->stream, &cap) != hipSuccess) direct = true;
    if (direct || cap != hipStreamCaptureStatusNone) {
        // profiled (every launch timed by events on the stream), the null
        // stream (no capture), or captured by the caller: no graph
        for (int64_t t = 0; t < nsteps; ++t) {
            c4m_status s = b->three_d ? launch_step3b(b) : launch_step(b);
            if (s != C4M_OK) return s;
        }
        for (auto* p : b->probs) problem_add_steps(p, nsteps);
        return C4M_OK;
    }
    // runs of up to GRAPH_STEPS steps captured once each as a HIP graph
    // (the stage launches of each step, or one node per step) and replayed
    int64_t left = nsteps;
    while (left > 0) {
        const int64_t len = std::min<int64_t>(left, GRAPH_STEPS);
        auto it = b->graphs.find(len);
        if (it == b->graphs.end()) {
            hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return set_error(C4M_EDEVICE, "hipStreamBeginCapture");
            c4m_status s = C4M_OK;
            for (int64_t t = 0; t < len && s == C4M_OK; ++t) s = b->three_d ? launch_step3b(b) : launch_step(b);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(b->stream, &g);
            if (s != C4M_OK) {
                if (g) (void)hipGraphDestroy(g);
                return s;
            }
            if (e != hipSuccess) return set_error(C4M_EDEVICE, "hipStreamEndCapture");
            hipGraphExec_t x = nullptr;
            e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(g);
                return set_error(C4M_EDEVICE, "hipGraphInstantiate");
            }
            it = b->graphs.emplace(len, std::make_pair(g, x)).first;
        }
        hipError_t e = hipGraphLaunch(it->second.second, b->stream);
        if (e != hipSuccess) return set_error(C4M_EDEVICE, "hipGraphLaunch");
        left -= len;
    }
    for (auto* p : b->probs) problem_add_steps(p, nsteps);
    return C4M_OK;
}

c4m_status c4m_batch_check(c4m_batch* b)
{
    if (!b) return set_error(C4M_EINVAL, "null batch");
    if (b->three_d) return C4M_OK;             // no stage waits in the 3D form
    int h = 0;
    hipError_t e = hipMemcpyAsync(&h, b->sched.err, sizeof(int), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return set_error(C4M_EDEVICE, hipGetErrorString(e));
    if (h) {
        e = hipMemsetAsync(b->sched.err, 0, sizeof(int), b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        return set_error(C4M_EDEVICE, "a stage wait of the batched step gave up (results of that call are invalid)");
    }
    return C4M_OK;
}

c4m_status c4m_batch_get_info(c4m_batch* b, c4m_info* info)
{
    if (!b || !info) return set_error(C4M_EINVAL, "null argument");
    c4m_status s = flush_batch_profile(b);
    if (s != C4M_OK) return s;
    memset(info, 0, sizeof(*info));
    c4m_info m{};
    for (auto* p : b->probs) {
        if (c4m_get_info(p, &m) != C4M_OK) continue;
        info->steps = m.steps;
        info->sweeps = m.sweeps;
        info->nonfinite |= m.nonfinite;
        info->workspace_bytes += m.workspace_bytes;
        for (int k = 0; k < C4M_K_COUNT; ++k) info->kernel_alg_bytes[k] += m.kernel_alg_bytes[k];
    }
    // one launch per step carries both half-steps of every member
    info->kernel_alg_bytes[C4M_K_STEP] = info->kernel_alg_bytes[C4M_K_STEP_E] + info->kernel_alg_bytes[C4M_K_STEP_H];
    for (int k = 0; k < C4M_K_COUNT; ++k) {
        info->kernel_ms[k] = b->kernel_ms[k];
        info->kernel_launches[k] = b->kernel_launches[k];
    }
    return C4M_OK;
}

c4m_status c4m_batch_destroy(c4m_batch* b)
{
    if (!b) return set_error(C4M_EINVAL, "null batch");
    (void)flush_batch_profile(b);
    for (hipEvent_t e : b->pool) (void)hipEventDestroy(e);
    for (auto& kv : b->graphs) {
        (void)hipGraphExecDestroy(kv.second.second);
        (void)hipGraphDestroy(kv.second.first);
    }
    if (b->owns)
        for (auto* p : b->probs) problem_destroy_owned(p);
    delete b;
    return C4M_OK;
}

}  // extern "C"
