// c4m_batch.hip -- batched form: many independent 2D TM cavity problems of
// uneven N advanced together.
//
// A step is five phases (Step 1 x-lines, Step 1 column solve, Step 2
// x-lines, Step 2 Hx and Hy column solves).  Each phase is ONE persistent
// launch over the work items (problem, tile) of every problem: workgroups
// take items from a device counter until the queue is empty, so problems of
// very different sizes share the machine without one launch per problem.
// The last workgroup to leave resets the counter for the next launch (no
// memset, so the step can be captured into a HIP graph and replayed).
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "c4m_stream_2d.h"

namespace c4m {

bool strip_form_2d(int shape, bool mixed, int sweeps);

// Strip shape of the batched form: the single-problem default (8 steps per
// unrolled block, one step of prefetch), so members equal problems run
// alone bit for bit.
constexpr int BS_U = 8, BS_LA = 1, BS_WPE = 3;

struct BatchProb {
    XArgs xe, xh;            // x-line arguments of Step 1 and Step 2
    ColArgs ce, chx, chy;    // column arguments of the three solves
    int tiles_x[5];          // tiles along x per phase
    int xtiles[5];           // x-line phases: tiles before the band-table items
    StripPlan plan[3];       // strip form: plans of the E, Hx and Hy solves
};

enum { PH_XE = 0, PH_CE = 1, PH_XH = 2, PH_CHX = 3, PH_CHY = 4, NPH = 5 };

struct PhaseQueue {
    const int* prefix;       // [count + 1] first work item of each problem
    int count;
    int* ctr;                // [0, NXCD): next item of each chunk, [NXCD]: workgroups finished
};
static_assert(NXCD + 1 <= 16, "the counters of a phase share one 64-byte line");

__device__ __forceinline__ int find_problem(const PhaseQueue& q, int item)
{
    int lo = 0, hi = q.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (q.prefix[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Claim the next item for the whole workgroup; -1 when the queue is empty.
// The item sequence is cut into NXCD contiguous chunks with one counter
// each.  Workgroup IDs are dealt to the XCDs in turn, so a workgroup takes
// items from the chunk of its XCD first and from the others once that is
// empty: the items an XCD runs at the same time are neighbours and share
// their halo data in that XCD's L2.
__device__ __forceinline__ int claim(const PhaseQueue& q, int total, int* slot)
{
    __syncthreads();                         // every thread has read the previous item
    if (threadIdx.x == 0) {
        const int per = (total + NXCD - 1) / NXCD;
        const int home = (int)(blockIdx.x % NXCD);
        int item = -1;
        for (int j = 0; j < NXCD && item < 0; ++j) {
            const int c = (home + j) % NXCD;
            const int len = min(per, total - c * per);
            if (len <= 0) continue;
            const int k = atomicAdd(q.ctr + c, 1);
            if (k < len) item = c * per + k;
        }
        *slot = item;
    }
    __syncthreads();
    return *slot;
}

// The last workgroup to leave resets the chunk counters and its own count.
__device__ __forceinline__ void finish(const PhaseQueue& q)
{
    if (threadIdx.x == 0) {
        __threadfence();
        const int done = atomicAdd(q.ctr + NXCD, 1);
        if (done == (int)gridDim.x - 1) {
            for (int c = 0; c < NXCD; ++c) atomicExch(q.ctr + c, 0);
            atomicExch(q.ctr + NXCD, 0);
        }
    }
}

// PF: Step 1 x-lines of the strip form (see k_xlines).
template <int MODE, bool PF>
__global__ __launch_bounds__(256) void k_batch_x(const BatchProb* __restrict__ bp, PhaseQueue q, int total,
                                                 int phase, Coef cf, PadeTaps taps)
{
    __shared__ int slot;
    for (;;) {
        const int it = claim(q, total, &slot);
        if (it < 0) break;
        const int p = find_problem(q, it);
        const int local = it - q.prefix[p];
        const int tx = bp[p].tiles_x[phase];
        const XArgs& xa = phase == PH_XE ? bp[p].xe : bp[p].xh;
        if (local >= bp[p].xtiles[phase]) {
            // band-table item of the following strip solve
            const int id = local - bp[p].xtiles[phase];
            const ColArgs& ca = phase == PH_XE ? bp[p].ce : bp[p].chx;
            const int nbx = (xa.N + 1 + 255) / 256, nbr = band_rows(xa.L);
            const int gx = (id % nbx) * 256 + (int)threadIdx.x, r = (id / nbx) % nbr, e = id / (nbx * nbr);
            if (MODE == XL_H_TRACKED)
                yband_entry<false>(ca.src, ca.yb, xa.N, xa.P, xa.L, gx, r, e);
            else
                yband_entry<true>(ca.src, ca.yb, xa.N, xa.P, xa.L, gx, r, e);
            continue;
        }
        if constexpr (MODE == XL_E_TRACKED || MODE == XL_E_DISCRETE)
            xlines_e_tile<MODE == XL_E_TRACKED, PF>(xa.src, xa.t0, xa.t1, xa.N, xa.P, xa.L, cf, local % tx, local / tx);
        else
            xlines_tile<MODE>(xa.src, xa.t0, xa.t1, xa.N, xa.P, xa.L, cf, taps, local % tx, local / tx);
    }
    finish(q);
}

template <int K, int MODE, class S, int FORM>
__global__ __launch_bounds__(S::NTC) __attribute__((amdgpu_waves_per_eu(S::NL == 4 ? 4 : 2))) void k_batch_col(
    const BatchProb* __restrict__ bp, PhaseQueue q, int total, int phase, Coef cf, PadeTaps taps,
    ChebSchedule cs)
{
    __shared__ int slot;
    for (;;) {
        const int it = claim(q, total, &slot);
        if (it < 0) break;
        const int p = find_problem(q, it);
        const int local = it - q.prefix[p];
        const int tx = bp[p].tiles_x[phase];
        const int ty = (q.prefix[p + 1] - q.prefix[p]) / tx;
        const ColArgs& ca = phase == PH_CE ? bp[p].ce : (phase == PH_CHX ? bp[p].chx : bp[p].chy);
        const PadeLine& L = phase == PH_CE ? bp[p].xe.L : bp[p].xh.L;
        col_tile<K, MODE, S, FORM>(ca, cf, taps, L, cs, local / ty, local % ty);   // y fastest
    }
    finish(q);
}

// Strip form: a workgroup claims four consecutive items, one per wave.
__device__ __forceinline__ int claim4(const PhaseQueue& q, int total, int* slot)
{
    __syncthreads();                         // every wave has read the previous items
    if (threadIdx.x == 0) {
        const int per = (total + NXCD - 1) / NXCD;
        const int home = (int)(blockIdx.x % NXCD);
        int item = -1, cnt = 0;
        for (int j = 0; j < NXCD && item < 0; ++j) {
            const int c = (home + j) % NXCD;
            const int len = min(per, total - c * per);
            if (len <= 0) continue;
            const int k = atomicAdd(q.ctr + c, SW_WAVES);
            if (k < len) {
                item = c * per + k;
                cnt = min(SW_WAVES, len - k);
            }
        }
        slot[0] = item;
        slot[1] = cnt;
    }
    __syncthreads();
    const int w = (int)(threadIdx.x / SW_COLS);
    const int base = slot[0], cnt = slot[1];
    if (base < 0) return -1;
    return w < cnt ? base + w : -2;         // -2: this wave idles this round
}

template <int K, int MODE>
__global__ __launch_bounds__(SW_COLS * SW_WAVES) __attribute__((amdgpu_waves_per_eu(BS_WPE))) void k_batch_strip(
    const BatchProb* __restrict__ bp, PhaseQueue q, int total, int phase, Coef cf, ChebSchedule cs)
{
    using SS = StripShape<K, MODE, BS_U, BS_LA>;
    __shared__ int slot[2];
    const int k = phase == PH_CE ? 0 : (phase == PH_CHX ? 1 : 2);
    for (;;) {
        const int got = claim4(q, total, slot);
        if (got == -1) break;
        if (got < 0) continue;
        const int it = __builtin_amdgcn_readfirstlane(got);
        const int p = find_problem(q, it);
        const int local = it - q.prefix[p];
        const ColArgs& ca = k == 0 ? bp[p].ce : (k == 1 ? bp[p].chx : bp[p].chy);
        const PadeLine& L = k == 0 ? bp[p].xe.L : bp[p].xh.L;
        int strip, y0, tr;
        bool up;
        bp[p].plan[k].item(local, strip, y0, tr, up);
        strip_tile<K, MODE, BS_U, BS_LA>(ca, cf, L, cs, ca.g.lo[0] + strip * SS::OW, y0, tr, up);
    }
    finish(q);
}

static int col_tiles_k(int K, int shape, bool mixed, const UGrid& g, int* tx)
{
    if (mixed)
        return with_k_mixed(K, [&]<int KK, class S>() {
            *tx = col_tiles_x<KK, S>(g);
            return col_tiles_x<KK, S>(g) * col_tiles_y<KK, S>(g);
        });
    return with_k_shape(K, shape, [&]<int KK, class S>() {
        *tx = col_tiles_x<KK, S>(g);
        return col_tiles_x<KK, S>(g) * col_tiles_y<KK, S>(g);
    });
}

// workgroups of a persistent launch: what fits on the device at once
template <class Kern>
static int resident_blocks(Kern kern, int threads)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, threads, 0) != hipSuccess || per < 1) per = 1;
    return cus * per;
}

template <int MODE>
static int blocks_x(bool strips)
{
    constexpr bool E = MODE == XL_E_TRACKED || MODE == XL_E_DISCRETE;
    return (E && strips) ? resident_blocks(k_batch_x<MODE, E>, 256) : resident_blocks(k_batch_x<MODE, false>, 256);
}

template <int MODE>
static int blocks_col(int K, int shape, bool mixed)
{
    if (mixed)
        return with_k_mixed(K, [&]<int KK, class S>() { return resident_blocks(k_batch_col<KK, MODE, S, FORM_MIXED>, S::NTC); });
    return with_k_shape(K, shape, [&]<int KK, class S>() { return resident_blocks(k_batch_col<KK, MODE, S, FORM_FP64>, S::NTC); });
}

// K (2 .. 8) as a template argument for the strip form
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

template <int MODE>
static int blocks_strip(int K)
{
    return with_k_bstrip(K, [&]<int KK>() { return resident_blocks(k_batch_strip<KK, MODE>, SW_COLS * SW_WAVES); });
}

// plan of one strip solve of a batch member (device wave slots as for a
// problem run alone)
template <int MODE>
static bool batch_plan(int K, const UGrid& g, const PadeLine& L, StripPlan& plan)
{
    return with_k_bstrip(K, [&]<int KK>() {
        using SS = StripShape<KK, MODE, BS_U, BS_LA>;
        const int blocks = resident_blocks(k_batch_strip<KK, MODE>, SW_COLS * SW_WAVES);
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        return strip_plan<SS, KK, BS_U>(g, L, blocks * SW_WAVES, cus * 4, plan);
    });
}

template <int MODE>
static hipError_t launch_bs(int K, hipStream_t st, int blocks, const BatchProb* bp, const PhaseQueue& q, int total,
                            int phase, const Coef& cf, const ChebSchedule& cs)
{
    const int g = std::max(1, std::min(blocks, (total + SW_WAVES - 1) / SW_WAVES));
    return with_k_bstrip(K, [&]<int KK>() {
        hipLaunchKernelGGL((k_batch_strip<KK, MODE>), dim3(g), dim3(SW_COLS * SW_WAVES), 0, st, bp, q, total, phase, cf,
                           cs);
        return hipGetLastError();
    });
}

template <int MODE>
static hipError_t launch_bx(hipStream_t st, int blocks, const BatchProb* bp, const PhaseQueue& q, int total,
                            int phase, const Coef& cf, const PadeTaps& taps, bool strips)
{
    const int g = std::max(1, std::min(blocks, total));
    constexpr bool E = MODE == XL_E_TRACKED || MODE == XL_E_DISCRETE;
    if (E && strips)
        hipLaunchKernelGGL((k_batch_x<MODE, E>), dim3(g), dim3(256), 0, st, bp, q, total, phase, cf, taps);
    else
        hipLaunchKernelGGL((k_batch_x<MODE, false>), dim3(g), dim3(256), 0, st, bp, q, total, phase, cf, taps);
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_bc(int K, int shape, bool mixed, hipStream_t st, int blocks, const BatchProb* bp,
                            const PhaseQueue& q, int total, int phase, const Coef& cf, const PadeTaps& taps,
                            const ChebSchedule& cs)
{
    const int g = std::max(1, std::min(blocks, total));
    if (mixed)
        return with_k_mixed(K, [&]<int KK, class S>() {
            hipLaunchKernelGGL((k_batch_col<KK, MODE, S, FORM_MIXED>), dim3(g), dim3(S::NTC), 0, st, bp, q, total, phase,
                               cf, taps, cs);
            return hipGetLastError();
        });
    return with_k_shape(K, shape, [&]<int KK, class S>() {
        hipLaunchKernelGGL((k_batch_col<KK, MODE, S, FORM_FP64>), dim3(g), dim3(S::NTC), 0, st, bp, q, total, phase, cf,
                           taps, cs);
        return hipGetLastError();
    });
}

}  // namespace c4m

using namespace c4m;

// Internal hooks of the single-problem runtime (c4m_host.hip).
namespace c4m {
c4m_status problem_view(c4m_problem* p, ProblemView* v);
c4m_status problem_prepare(c4m_problem* p);     // carried-Laplacian conversion before stepping
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
    int* d_prefix = nullptr;       // [NPH][count + 1]
    int* d_ctr = nullptr;          // [NPH][16]: chunk counters and the finished count (64 bytes a phase)
    int total[NPH] = {};
    Coef coef{};
    PadeTaps taps_xe{}, taps_xh{};
    ChebSchedule cheb{};
    int blocks[NPH] = {};           // workgroups of each persistent launch
    bool owns = true;               // problems created by (and destroyed with) the batch
    bool strips = false;            // solves in the strip form
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

c4m_status check_uniform(const c4m_config* cfgs, int32_t count)
{
    if (!cfgs || count < 1) return set_error(C4M_EINVAL, "empty batch");
    for (int i = 0; i < count; ++i) {
        const c4m_config& c = cfgs[i];
        if (c.dim != 2) return set_error(C4M_EINVAL, "batched form takes 2D problems");
        if (c.solver != C4M_SOLVER_CHEBYSHEV)
            return set_error(C4M_EINVAL, "batched form runs the fused Chebyshev solve only");
        if (c.cfl != cfgs[0].cfl || c.z != cfgs[0].z || c.closure != cfgs[0].closure ||
            c.lap_mode != cfgs[0].lap_mode || c.precision != cfgs[0].precision ||
            c.solver != cfgs[0].solver || c.sweeps != cfgs[0].sweeps || c.tile_x != cfgs[0].tile_x ||
            c.tile_y != cfgs[0].tile_y)
            return set_error(C4M_EINVAL, "batched problems must share cfl, z, closure, lap_mode, precision, solver");
        size_t b = 0;
        c4m_status s = c4m_workspace_bytes(&c, &b);
        if (s != C4M_OK) return s;
    }
    return C4M_OK;
}

size_t tables_bytes(int count)
{
    return a256(sizeof(BatchProb) * count) + a256(sizeof(int) * NPH * (count + 1)) + a256(NPH * 64);
}

c4m_status launch_step(c4m_batch* b)
{
    const bool tracked = b->base.lap_mode == C4M_LAP_TRACKED;
    const bool mixed = b->base.precision == C4M_FP32_REFINED;
    const int K = b->cheb.sweeps;
    hipError_t e = hipSuccess;
    for (int ph = 0; ph < NPH && e == hipSuccess; ++ph) {
        if (!b->total[ph]) continue;
        PhaseQueue q{b->d_prefix + ph * (b->count + 1), b->count, b->d_ctr + ph * 16};
        const BatchProb* bp = b->d_probs;
        const int nb = b->blocks[ph];
        const int tot = b->total[ph];
        switch (ph) {
            case PH_XE:
                e = tracked ? launch_bx<XL_E_TRACKED>(b->stream, nb, bp, q, tot, ph, b->coef, b->taps_xe, b->strips)
                            : launch_bx<XL_E_DISCRETE>(b->stream, nb, bp, q, tot, ph, b->coef, b->taps_xe, b->strips);
                break;
            case PH_CE:
                if (b->strips) {
                    e = tracked ? launch_bs<COL_E_TRACKED>(K, b->stream, nb, bp, q, tot, ph, b->coef, b->cheb)
                                : launch_bs<COL_E_DISCRETE>(K, b->stream, nb, bp, q, tot, ph, b->coef, b->cheb);
                    break;
                }
                e = tracked ? launch_bc<COL_E_TRACKED>(K, b->base.tile_x, mixed, b->stream, nb, bp, q, tot, ph, b->coef, b->taps_xe, b->cheb)
                            : launch_bc<COL_E_DISCRETE>(K, b->base.tile_x, mixed, b->stream, nb, bp, q, tot, ph, b->coef, b->taps_xe, b->cheb);
                break;
            case PH_XH:
                e = tracked ? launch_bx<XL_H_TRACKED>(b->stream, nb, bp, q, tot, ph, b->coef, b->taps_xh, b->strips)
                            : launch_bx<XL_H_DISCRETE>(b->stream, nb, bp, q, tot, ph, b->coef, b->taps_xh, b->strips);
                break;
            case PH_CHX:
                if (b->strips) {
                    e = tracked ? launch_bs<COL_HX_TRACKED>(K, b->stream, nb, bp, q, tot, ph, b->coef, b->cheb)
                                : launch_bs<COL_HX_DISCRETE>(K, b->stream, nb, bp, q, tot, ph, b->coef, b->cheb);
                    break;
                }
                e = tracked ? launch_bc<COL_HX_TRACKED>(K, b->base.tile_x, mixed, b->stream, nb, bp, q, tot, ph, b->coef, b->taps_xh, b->cheb)
                            : launch_bc<COL_HX_DISCRETE>(K, b->base.tile_x, mixed, b->stream, nb, bp, q, tot, ph, b->coef, b->taps_xh, b->cheb);
                break;
            default:
                e = b->strips ? launch_bs<COL_HY>(K, b->stream, nb, bp, q, tot, ph, b->coef, b->cheb)
                              : launch_bc<COL_HY>(K, b->base.tile_x, mixed, b->stream, nb, bp, q, tot, ph, b->coef,
                                                  b->taps_xh, b->cheb);
                break;
        }
    }
    return e == hipSuccess ? C4M_OK : set_error(C4M_EDEVICE, hipGetErrorString(e));
}

}  // namespace

extern "C" {

c4m_status c4m_batch_workspace_bytes(const c4m_config* cfgs, int32_t count, size_t* bytes)
{
    c4m_status s = check_uniform(cfgs, count);
    if (s != C4M_OK) return s;
    if (!bytes) return set_error(C4M_EINVAL, "null bytes");
    size_t tot = tables_bytes(count);
    for (int i = 0; i < count; ++i) {
        size_t b = 0;
        c4m_workspace_bytes(&cfgs[i], &b);
        tot += a256(b);
    }
    *bytes = tot;
    return C4M_OK;
}

}  // extern "C"

namespace {

// Work-queue tables of a batch over b->probs, carved at `cur`.
c4m_status build_tables(c4m_batch* b, char* cur)
{
    const int count = b->count;
    b->d_probs = (BatchProb*)cur;
    cur += a256(sizeof(BatchProb) * count);
    b->d_prefix = (int*)cur;
    cur += a256(sizeof(int) * NPH * (count + 1));
    b->d_ctr = (int*)cur;
    std::vector<BatchProb> hp(count);
    std::vector<int> prefix((size_t)NPH * (count + 1), 0);
    const int shape = b->base.tile_x;
    const bool mixed = b->base.precision == C4M_FP32_REFINED;
    {
        // the strip form when every member's workspace fits one buffer resource
        ProblemView v0{};
        problem_view(b->probs[0], &v0);
        b->strips = strip_form_2d(shape, mixed, v0.cheb.sweeps);
        for (int i = 0; i < count && b->strips; ++i) {
            ProblemView v{};
            problem_view(b->probs[i], &v);
            if (!v.yband || v.used >= (size_t)0xFFFFF000u) b->strips = false;
        }
    }
    for (int i = 0; i < count; ++i) {
        ProblemView v{};
        problem_view(b->probs[i], &v);
        const int N = v.N;
        const bool tracked = b->base.lap_mode == C4M_LAP_TRACKED;
        BatchProb& d = hp[i];
        d.xe = XArgs{v.f[C4M_HY], v.tmp[0], v.tmp[1], N, v.P, v.line[1]};
        d.xh = XArgs{tracked ? v.ge[2] : v.f[C4M_EZ], v.tmp[0], v.tmp[1], N, v.P, v.line[0]};
        d.ce = ColArgs{v.f[C4M_HX], v.tmp[0], v.tmp[1], v.f[C4M_EZ], v.ge[2], ugrid_ez(N), N, v.P};
        d.chx = ColArgs{tracked ? v.ge[2] : v.f[C4M_EZ], nullptr, nullptr, v.f[C4M_HX], nullptr, ugrid_hx(N), N, v.P};
        d.chy = ColArgs{nullptr, v.tmp[1], nullptr, v.f[C4M_HY], nullptr, ugrid_hy(N), N, v.P};
        const int K = v.cheb.sweeps;
        int tiles[NPH];
        d.tiles_x[PH_XE] = xe_tiles_x(v.line[1].n_out);
        d.xtiles[PH_XE] = d.tiles_x[PH_XE] * xe_tiles_y(N);
        d.tiles_x[PH_XH] = xlines_tiles_x(v.line[0].n_out);
        d.xtiles[PH_XH] = d.tiles_x[PH_XH] * xlines_tiles_y(N);
        tiles[PH_XE] = d.xtiles[PH_XE];
        tiles[PH_XH] = d.xtiles[PH_XH];
        if (b->strips) {
            d.ce.yb = d.chx.yb = d.chy.yb = v.yband;
            const int nbx = (N + 1 + 255) / 256;
            tiles[PH_XE] += nbx * band_rows(v.line[1]) * 2;
            tiles[PH_XH] += nbx * band_rows(v.line[0]) * 2;
            bool ok = tracked ? batch_plan<COL_E_TRACKED>(K, d.ce.g, v.line[1], d.plan[0])
                              : batch_plan<COL_E_DISCRETE>(K, d.ce.g, v.line[1], d.plan[0]);
            ok = ok && (tracked ? batch_plan<COL_HX_TRACKED>(K, d.chx.g, v.line[0], d.plan[1])
                                : batch_plan<COL_HX_DISCRETE>(K, d.chx.g, v.line[0], d.plan[1]));
            ok = ok && batch_plan<COL_HY>(K, d.chy.g, v.line[0], d.plan[2]);
            if (!ok) return set_error(C4M_EINVAL, "no strip plan for a batch member");
            tiles[PH_CE] = d.plan[0].items();
            tiles[PH_CHX] = d.plan[1].items();
            tiles[PH_CHY] = d.plan[2].items();
        } else {
            tiles[PH_CE] = col_tiles_k(K, shape, mixed, d.ce.g, &d.tiles_x[PH_CE]);
            tiles[PH_CHX] = col_tiles_k(K, shape, mixed, d.chx.g, &d.tiles_x[PH_CHX]);
            tiles[PH_CHY] = col_tiles_k(K, shape, mixed, d.chy.g, &d.tiles_x[PH_CHY]);
        }
        for (int ph = 0; ph < NPH; ++ph)
            prefix[(size_t)ph * (count + 1) + i + 1] = prefix[(size_t)ph * (count + 1) + i] + tiles[ph];
        if (i == 0) {
            b->coef = v.coef;
            b->taps_xe = v.taps[1];
            b->taps_xh = v.taps[0];
            b->cheb = v.cheb;
        }
    }
    for (int ph = 0; ph < NPH; ++ph) b->total[ph] = prefix[(size_t)ph * (count + 1) + count];
    {
        const bool tracked = b->base.lap_mode == C4M_LAP_TRACKED;
        const int K = b->cheb.sweeps;
        b->blocks[PH_XE] = tracked ? blocks_x<XL_E_TRACKED>(b->strips) : blocks_x<XL_E_DISCRETE>(b->strips);
        b->blocks[PH_XH] = tracked ? blocks_x<XL_H_TRACKED>(b->strips) : blocks_x<XL_H_DISCRETE>(b->strips);
        if (b->strips) {
            b->blocks[PH_CE] = tracked ? blocks_strip<COL_E_TRACKED>(K) : blocks_strip<COL_E_DISCRETE>(K);
            b->blocks[PH_CHX] = tracked ? blocks_strip<COL_HX_TRACKED>(K) : blocks_strip<COL_HX_DISCRETE>(K);
            b->blocks[PH_CHY] = blocks_strip<COL_HY>(K);
        } else {
            b->blocks[PH_CE] = tracked ? blocks_col<COL_E_TRACKED>(K, shape, mixed) : blocks_col<COL_E_DISCRETE>(K, shape, mixed);
            b->blocks[PH_CHX] = tracked ? blocks_col<COL_HX_TRACKED>(K, shape, mixed) : blocks_col<COL_HX_DISCRETE>(K, shape, mixed);
            b->blocks[PH_CHY] = blocks_col<COL_HY>(K, shape, mixed);
        }
        const int mult = b->base.tile_y > 0 ? b->base.tile_y : 1;   // persistent grid multiplier
        for (int ph = 0; ph < NPH; ++ph) b->blocks[ph] *= mult;
    }
    hipError_t e = hipMemcpyAsync(b->d_probs, hp.data(), sizeof(BatchProb) * count, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_prefix, prefix.data(), sizeof(int) * prefix.size(), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_ctr, 0, NPH * 64, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    return e == hipSuccess ? C4M_OK : set_error(C4M_EDEVICE, hipGetErrorString(e));
}

}  // namespace

extern "C" {

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
    c4m_batch* b = new (std::nothrow) c4m_batch();
    if (!b) return set_error(C4M_ENOMEM, "host allocation");
    b->count = count;
    b->base = cfgs[0];
    b->stream = (hipStream_t)hip_stream;
    char* tables = (char*)d_workspace;
    char* cur = tables + tables_bytes(count);
    for (int i = 0; i < count && s == C4M_OK; ++i) {
        size_t pb = 0;
        c4m_workspace_bytes(&cfgs[i], &pb);
        c4m_problem* p = nullptr;
        s = problem_create_owned(&cfgs[i], cur, pb, b->stream, &p);
        if (s != C4M_OK) break;
        cur += a256(pb);
        b->probs.push_back(p);
    }
    if (s == C4M_OK) s = build_tables(b, tables);
    if (s != C4M_OK) {
        for (auto* p : b->probs) problem_destroy_owned(p);
        delete b;
        return s;
    }
    *out = b;
    return C4M_OK;
}

c4m_status c4m_batch_tables_bytes(int32_t count, size_t* bytes)
{
    if (count < 1 || !bytes) return set_error(C4M_EINVAL, "bad count");
    *bytes = tables_bytes(count);
    return C4M_OK;
}

c4m_status c4m_batch_create_from(c4m_problem* const* probs, int32_t count, void* d_tables, size_t bytes,
                                 void* hip_stream, c4m_batch** out)
{
    if (!out || !probs || count < 1) return set_error(C4M_EINVAL, "bad arguments");
    *out = nullptr;
    if (!d_tables || ((uintptr_t)d_tables & 255)) return set_error(C4M_EINVAL, "tables must be 256-byte aligned");
    if (bytes < tables_bytes(count)) return set_error(C4M_ENOMEM, "table space smaller than c4m_batch_tables_bytes");
    std::vector<c4m_config> cfgs(count);
    for (int i = 0; i < count; ++i) {
        if (!probs[i]) return set_error(C4M_EINVAL, "null problem");
        cfgs[i] = *problem_config(probs[i]);
    }
    c4m_status s = check_uniform(cfgs.data(), count);
    if (s != C4M_OK) return s;
    c4m_batch* b = new (std::nothrow) c4m_batch();
    if (!b) return set_error(C4M_ENOMEM, "host allocation");
    b->count = count;
    b->base = cfgs[0];
    b->stream = (hipStream_t)hip_stream;
    b->owns = false;
    b->probs.assign(probs, probs + count);
    s = build_tables(b, (char*)d_tables);
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
    for (auto* p : b->probs) {
        c4m_status s = problem_prepare(p);
        if (s != C4M_OK) return s;
    }
    if (nsteps == 0) return C4M_OK;
    // one step captured once as a graph, then replayed
    if (!b->exec) {
        hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return set_error(C4M_EDEVICE, "hipStreamBeginCapture");
        c4m_status s = launch_step(b);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->stream, &g);
        if (s != C4M_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess) return set_error(C4M_EDEVICE, "hipStreamEndCapture");
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            b->exec = nullptr;
            return set_error(C4M_EDEVICE, "hipGraphInstantiate");
        }
        b->graph = g;
    }
    for (int64_t t = 0; t < nsteps; ++t) {
        hipError_t e = hipGraphLaunch(b->exec, b->stream);
        if (e != hipSuccess) return set_error(C4M_EDEVICE, "hipGraphLaunch");
    }
    for (auto* p : b->probs) problem_add_steps(p, nsteps);
    return C4M_OK;
}

c4m_status c4m_batch_destroy(c4m_batch* b)
{
    if (!b) return set_error(C4M_EINVAL, "null batch");
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->owns)
        for (auto* p : b->probs) problem_destroy_owned(p);
    delete b;
    return C4M_OK;
}

}  // extern "C"
