// c4m_kernels_2d.hip -- single-problem launches of the 2D TM kernels (the
// tile code lives in c4m_tiles_2d.h and is shared with the batched form).
#include <map>
#include <mutex>
#include <tuple>

#include "c4m_stream_2d.h"

namespace c4m {

// Band rows of the strip form's y-lines, computed by extra workgroups of
// the x-line launch that precedes each strip solve.
struct YbandArgs {
    const double* src;      // y-line source of the following solve
    double* yb;             // band table (null: no band work)
    PadeLine L;
    int split;              // conditioned derivatives as well
};
__host__ __device__ inline int yband_blocks(const YbandArgs& y, int N)
{
    return y.yb ? ((N + 1 + 255) / 256) * band_rows(y.L) * 2 : 0;
}

// Step 1 x-lines take the raw-derivative tiles (xlines_e_tile), Step 2
// the direct ones.
template <int MODE>
__host__ __device__ inline int xl_tiles_x(int n_out)
{
    return (MODE == XL_E_TRACKED || MODE == XL_E_DISCRETE) ? xe_tiles_x(n_out) : xlines_tiles_x(n_out);
}
template <int MODE>
__host__ __device__ inline int xl_tiles_y(int N)
{
    return (MODE == XL_E_TRACKED || MODE == XL_E_DISCRETE) ? xe_tiles_y(N) : xlines_tiles_y(N);
}

// PF: Step 1 x-lines of the strip form (raw derivative on every row, T0 on
// the band columns only; the strips form the rest of T0).
template <int MODE, bool PF = false>
__global__ __launch_bounds__(256) void k_xlines(XArgs xa, Coef cf, PadeTaps taps, YbandArgs yba)
{
    constexpr bool E = MODE == XL_E_TRACKED || MODE == XL_E_DISCRETE;
    __shared__ double lds[E ? XE_LDS : xt_lds(MODE)];
    const int ntx = xl_tiles_x<MODE>(xa.L.n_out), nty = xl_tiles_y<MODE>(xa.N);
    const int xgrid = xcd_grid(ntx * nty);
    if ((int)blockIdx.x >= xgrid) {
        const int id = (int)blockIdx.x - xgrid, nbx = (xa.N + 1 + 255) / 256, nbr = band_rows(yba.L);
        const int bx = id % nbx, r = (id / nbx) % nbr, e = id / (nbx * nbr);
        const int gx = bx * 256 + (int)threadIdx.x;
        if (yba.split)
            yband_entry<true>(yba.src, yba.yb, xa.N, xa.P, yba.L, gx, r, e);
        else
            yband_entry<false>(yba.src, yba.yb, xa.N, xa.P, yba.L, gx, r, e);
        return;
    }
    int l;
    if (!xcd_tile(ntx * nty, l)) return;
    if constexpr (MODE == XL_E_TRACKED || MODE == XL_E_DISCRETE)
        xlines_e_tile<MODE == XL_E_TRACKED, PF>(xa.src, xa.t0, xa.t1, xa.N, xa.P, xa.L, cf, l % ntx, l / ntx, lds);
    else
        xlines_tile<MODE>(xa.src, xa.t0, xa.t1, xa.N, xa.P, xa.L, cf, taps, l % ntx, l / ntx, lds);
}

template <int K, int MODE, class S, int FORM>
__global__ __launch_bounds__(S::NTC) __attribute__((amdgpu_waves_per_eu(S::NL == 4 ? 4 : 2))) void k_col(
    ColArgs a, Coef cf, PadeTaps taps, PadeLine L, ChebSchedule cs)
{
    const int ntx = col_tiles_x<K, S>(a.g), nty = col_tiles_y<K, S>(a.g);
    int l;
    if (!xcd_tile(ntx * nty, l)) return;
    col_tile<K, MODE, S, FORM>(a, cf, taps, L, cs, l / nty, l % nty);   // y fastest
}

template <int K, int MODE, int U, int LA, int WPE>
__global__ __launch_bounds__(SW_COLS * SW_WAVES) __attribute__((amdgpu_waves_per_eu(WPE))) void k_strip(
    ColArgs a, Coef cf, PadeLine L, ChebSchedule cs, StripPlan plan)
{
    using SS = StripShape<K, MODE, U, LA>;
    const int items = plan.items();
    int l;
    if (!xcd_tile((items + SW_WAVES - 1) / SW_WAVES, l)) return;
    // the wave index is uniform over the wave: say so, so that everything
    // derived from it (rows, offsets, table rows) lives in scalar registers
    const int item = l * SW_WAVES + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / SW_COLS));
    if (item >= items) return;
    int strip, y0, tr;
    bool up;
    plan.item(item, strip, y0, tr, up);
    strip_tile<K, MODE, U, LA>(a, cf, L, cs, a.g.lo[0] + strip * SS::OW, y0, tr, up);
}

// Step 2 in the strip form: the Hx strips (mode MA) and the Hy strips of a
// step in one launch.  The Hx items come first; each part keeps the
// XCD-aware order over its own items (the part sizes are whole rounds of
// the XCD count), so the Hy items fill the device as the Hx items drain.
template <int K, int MA, int U, int LA, int WPE>
__global__ __launch_bounds__(SW_COLS * SW_WAVES) __attribute__((amdgpu_waves_per_eu(WPE))) void k_strip_h(
    ColArgs a, ColArgs b, Coef cf, PadeLine L, ChebSchedule cs, StripPlan pa, StripPlan pb)
{
    using SA = StripShape<K, MA, U, LA>;
    using SB = StripShape<K, COL_HY, U, LA>;
    const int na = pa.items(), nb = pb.items();
    const int ga = xcd_grid((na + SW_WAVES - 1) / SW_WAVES);
    const bool first = (int)blockIdx.x < ga;
    const int tiles = first ? (na + SW_WAVES - 1) / SW_WAVES : (nb + SW_WAVES - 1) / SW_WAVES;
    const int per = (tiles + NXCD - 1) / NXCD;
    const int g = (int)blockIdx.x - (first ? 0 : ga);
    const int l = (g % NXCD) * per + g / NXCD;
    if (l >= tiles) return;
    const int item = l * SW_WAVES + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / SW_COLS));
    int strip, y0, tr;
    bool up;
    if (first) {
        if (item >= na) return;
        pa.item(item, strip, y0, tr, up);
        strip_tile<K, MA, U, LA>(a, cf, L, cs, a.g.lo[0] + strip * SA::OW, y0, tr, up);
    } else {
        if (item >= nb) return;
        pb.item(item, strip, y0, tr, up);
        strip_tile<K, COL_HY, U, LA>(b, cf, L, cs, b.g.lo[0] + strip * SB::OW, y0, tr, up);
    }
}

// Whether a 2D single-problem solve takes the strip form (the host then
// provides the band table, in a workspace whose span fits one buffer).
bool strip_form_2d(int shape, bool mixed, int sweeps)
{
    return (shape == 0 || shape == 4) && !mixed && sweeps >= 2 && sweeps <= MAX_SWEEPS;
}

// Dispatch a callable templated on K (2 .. 8) for the strip form.
template <class F>
inline hipError_t with_k_strip(int K, F&& f)
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

template <int K, int MODE, int U, int LA, int WPE>
static hipError_t launch_strip(hipStream_t st, const ColArgs& a, const Coef& cf, const PadeLine& L,
                               const ChebSchedule& cs)
{
    using SS = StripShape<K, MODE, U, LA>;
    auto kern = k_strip<K, MODE, U, LA, WPE>;
    // plans of this kernel per problem geometry, made on first use
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int, int, int>, StripPlan> plans;
    const StripPlan* plan = nullptr;
    {
        std::lock_guard<std::mutex> lock(mu);
        const auto key = std::make_tuple(a.N, a.g.lo[0], a.g.hi[0], a.g.lo[1], a.g.hi[1], L.n_in);
        auto it = plans.find(key);
        if (it == plans.end()) {
            int dev = 0, cus = 0, blocks = 0;
            (void)hipGetDevice(&dev);
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kern, SW_COLS * SW_WAVES, 0);
            const int slots = (cus > 0 ? cus : 256) * (blocks > 0 ? blocks : 1) * SW_WAVES;
            StripPlan pl{};
            if (!strip_plan<SS, K, U>(a.g, L, slots, (cus > 0 ? cus : 256) * 4, pl)) return hipErrorInvalidValue;
            it = plans.emplace(key, pl).first;
        }
        plan = &it->second;
    }
    const dim3 grid(xcd_grid((plan->items() + SW_WAVES - 1) / SW_WAVES));
    hipLaunchKernelGGL(kern, grid, dim3(SW_COLS * SW_WAVES), 0, st, a, cf, L, cs, *plan);
    return hipGetLastError();
}

// Step 2 strips in one launch (k_strip_h); each part is planned for
// 1 / STRIP_H_DIV of the resident wave slots.
constexpr int STRIP_H_DIV = 2;
template <int K, int MA, int U, int LA, int WPE>
static hipError_t launch_strip_h(hipStream_t st, const ColArgs& a, const ColArgs& b, const Coef& cf,
                                 const PadeLine& L, const ChebSchedule& cs)
{
    using SA = StripShape<K, MA, U, LA>;
    using SB = StripShape<K, COL_HY, U, LA>;
    auto kern = k_strip_h<K, MA, U, LA, WPE>;
    static std::mutex mu;
    static std::map<std::tuple<int, int, int>, std::pair<StripPlan, StripPlan>> plans;
    const std::pair<StripPlan, StripPlan>* pl = nullptr;
    {
        std::lock_guard<std::mutex> lock(mu);
        int dev = 0;
        (void)hipGetDevice(&dev);
        const auto key = std::make_tuple(dev, a.N, L.n_in);
        auto it = plans.find(key);
        if (it == plans.end()) {
            int cus = 0, blocks = 0;
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kern, SW_COLS * SW_WAVES, 0);
            cus = cus > 0 ? cus : 256;
            const int slots = cus * (blocks > 0 ? blocks : 1) * SW_WAVES;
            std::pair<StripPlan, StripPlan> pp{};
            if (!strip_plan<SA, K, U>(a.g, L, slots / STRIP_H_DIV, cus * 4, pp.first) ||
                !strip_plan<SB, K, U>(b.g, L, slots / STRIP_H_DIV, cus * 4, pp.second))
                return hipErrorInvalidValue;
            it = plans.emplace(key, pp).first;
        }
        pl = &it->second;
    }
    const int ga = xcd_grid((pl->first.items() + SW_WAVES - 1) / SW_WAVES);
    const int gb = xcd_grid((pl->second.items() + SW_WAVES - 1) / SW_WAVES);
    hipLaunchKernelGGL(kern, dim3(ga + gb), dim3(SW_COLS * SW_WAVES), 0, st, a, b, cf, L, cs, pl->first, pl->second);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <int MODE>
static hipError_t launch_col(int shape, bool mixed, hipStream_t st, const ColArgs& a, const Coef& cf,
                             const PadeTaps& taps, const PadeLine& L, const ChebSchedule& cs)
{
    if (mixed)
        return with_k_mixed(cs.sweeps, [&]<int K, class S>() {
            const dim3 grid(xcd_grid(col_tiles_x<K, S>(a.g) * col_tiles_y<K, S>(a.g)));
            hipLaunchKernelGGL((k_col<K, MODE, S, FORM_MIXED>), grid, dim3(S::NTC), 0, st, a, cf, taps, L, cs);
            return hipGetLastError();
        });
    // shape 0 (default) and 4: the strip form where it applies (the caller
    // passes the band table only then); 1, 2, 3: the column tiles (64 x 4,
    // 128 x 2, 128 x 4 lanes)
    if (strip_form_2d(shape, mixed, cs.sweeps) && a.yb)
        return with_k_strip(cs.sweeps, [&]<int K>() {
            if (shape == 0) return launch_strip<K, MODE, 8, 1, 3>(st, a, cf, L, cs);
            return launch_strip<K, MODE, 16, 1, 3>(st, a, cf, L, cs);
        });
    return with_k_shape(cs.sweeps, shape, [&]<int K, class S>() {
        const dim3 grid(xcd_grid(col_tiles_x<K, S>(a.g) * col_tiles_y<K, S>(a.g)));
        hipLaunchKernelGGL((k_col<K, MODE, S, FORM_FP64>), grid, dim3(S::NTC), 0, st, a, cf, taps, L, cs);
        return hipGetLastError();
    });
}

// Right-hand side only (no solve halo): b on the unknowns, and the raw curl
// for the G_E update with the carried Laplacian.
template <int MODE>
static hipError_t launch_col_rhs(hipStream_t st, const ColArgs& a, const Coef& cf, const PadeTaps& taps,
                                 const PadeLine& L, const ChebSchedule& cs)
{
    const dim3 grid(xcd_grid(col_tiles_x<0, Shape0>(a.g) * col_tiles_y<0, Shape0>(a.g)));
    hipLaunchKernelGGL((k_col<0, MODE, Shape0, FORM_RHS>), grid, dim3(Shape0::NTC), 0, st, a, cf, taps, L, cs);
    return hipGetLastError();
}

hipError_t launch_rhs_e_2d(hipStream_t st, bool tracked, const double* hx, const double* hy, double* t0,
                           double* t1, int N, int P, const Coef& cf, const PadeTaps& taps,
                           const PadeLine& line_h2n, double* yb)
{
    // x-lines of Hy: N inputs, N-1 outputs, rows 1..N-1; with the strip
    // form also the band rows of the y-lines of Hx
    const YbandArgs yba{hx, yb, line_h2n, 1};
    const dim3 grid(xcd_grid(xe_tiles_x(line_h2n.n_out) * xe_tiles_y(N)) + yband_blocks(yba, N));
    const XArgs xa{hy, t0, t1, N, P, line_h2n};
    if (yb && tracked)
        hipLaunchKernelGGL((k_xlines<XL_E_TRACKED, true>), grid, dim3(256), 0, st, xa, cf, taps, yba);
    else if (yb)
        hipLaunchKernelGGL((k_xlines<XL_E_DISCRETE, true>), grid, dim3(256), 0, st, xa, cf, taps, yba);
    else if (tracked)
        hipLaunchKernelGGL(k_xlines<XL_E_TRACKED>, grid, dim3(256), 0, st, xa, cf, taps, yba);
    else
        hipLaunchKernelGGL(k_xlines<XL_E_DISCRETE>, grid, dim3(256), 0, st, xa, cf, taps, yba);
    return hipGetLastError();
}

hipError_t launch_solve_e_2d(hipStream_t st, int shape, bool mixed, bool tracked, const double* hx, double* ez, double* ge,
                             const double* t0, const double* t1, int N, int P, const Coef& cf,
                             const PadeTaps& taps, const PadeLine& line_h2n, const ChebSchedule& cs, double* yb)
{
    ColArgs a{hx, t0, t1, ez, ge, ugrid_ez(N), N, P};
    a.yb = yb;
    if (tracked) return launch_col<COL_E_TRACKED>(shape, mixed, st, a, cf, taps, line_h2n, cs);
    return launch_col<COL_E_DISCRETE>(shape, mixed, st, a, cf, taps, line_h2n, cs);
}

hipError_t launch_rhs_h_2d(hipStream_t st, bool tracked, const double* src, double* t0, double* t1,
                           int N, int P, const Coef& cf, const PadeTaps& taps,
                           const PadeLine& line_n2h, double* yb)
{
    // x-lines of G_E: N+1 inputs, N outputs (Hy half points), rows 1..N-1;
    // with the strip form also the band rows of the y-lines of the same source
    const YbandArgs yba{src, yb, line_n2h, tracked ? 0 : 1};
    const dim3 grid(xcd_grid(xlines_tiles_x(line_n2h.n_out) * xlines_tiles_y(N)) + yband_blocks(yba, N));
    const XArgs xa{src, t0, t1, N, P, line_n2h};
    if (tracked)
        hipLaunchKernelGGL(k_xlines<XL_H_TRACKED>, grid, dim3(256), 0, st, xa, cf, taps, yba);
    else
        hipLaunchKernelGGL(k_xlines<XL_H_DISCRETE>, grid, dim3(256), 0, st, xa, cf, taps, yba);
    return hipGetLastError();
}

hipError_t launch_solve_h_2d(hipStream_t st, int shape, bool mixed, bool tracked, const double* src, double* hx, double* hy,
                             const double* t1, int N, int P, const Coef& cf, const PadeTaps& taps,
                             const PadeLine& line_n2h, const ChebSchedule& cs, double* yb)
{
    // Hx: Dirichlet in x (nodes 1..N-1), Neumann in y (half points 0..N-1);
    // right-hand side -(1/Z) delta_y G_E along columns
    ColArgs ax{src, nullptr, nullptr, hx, nullptr, ugrid_hx(N), N, P};
    ax.yb = yb;
    // Hy: Neumann in x, Dirichlet in y; right-hand side T1 from the x-lines
    ColArgs ay{nullptr, t1, nullptr, hy, nullptr, ugrid_hy(N), N, P};
    ay.yb = yb;
    if (shape == 0 && strip_form_2d(shape, mixed, cs.sweeps) && yb)
        return with_k_strip(cs.sweeps, [&]<int K>() {
            return tracked ? launch_strip_h<K, COL_HX_TRACKED, 8, 1, 3>(st, ax, ay, cf, line_n2h, cs)
                           : launch_strip_h<K, COL_HX_DISCRETE, 8, 1, 3>(st, ax, ay, cf, line_n2h, cs);
        });
    hipError_t e = tracked ? launch_col<COL_HX_TRACKED>(shape, mixed, st, ax, cf, taps, line_n2h, cs)
                           : launch_col<COL_HX_DISCRETE>(shape, mixed, st, ax, cf, taps, line_n2h, cs);
    if (e != hipSuccess) return e;
    return launch_col<COL_HY>(shape, mixed, st, ay, cf, taps, line_n2h, cs);
}

// PCG forms of the two solves.  Temporaries: pt[0] x, pt[1] r (= b),
// pt[2], pt[3] search directions, pt[4] M p, pt[5] 1/diag(M), pt[6] z.
static PcgArgs pcg_args(double* const* pt, const UGrid& g, int P, const Coef& cf, double* part, PcgState* pst,
                        double rtol)
{
    PcgArgs a{};
    a.x = pt[0];
    a.r = pt[1];
    a.p[0] = pt[2];
    a.p[1] = pt[3];
    a.q = pt[4];
    a.dinv = pt[5];
    a.z = pt[6];
    a.part = part;
    a.st = pst;
    a.g = g;
    a.P = P;
    a.plane = 0;
    a.alpha = cf.alpha;
    a.beta = cf.beta;
    a.rtol2 = rtol * rtol;
    return a;
}

hipError_t launch_pcg_e_2d(hipStream_t st, bool tracked, const double* hx, double* ez, double* ge,
                           const double* t0, double* t1, int N, int P, const Coef& cf, const PadeTaps& taps,
                           const PadeLine& line_h2n, const ChebSchedule& cs, double* const* pt, double* part,
                           PcgState* pst, double rtol, int max_iter)
{
    ColArgs a{hx, t0, t1, ez, ge, ugrid_ez(N), N, P, pt[1], t1};
    hipError_t e = tracked ? launch_col_rhs<COL_E_TRACKED>(st, a, cf, taps, line_h2n, cs)
                           : launch_col_rhs<COL_E_DISCRETE>(st, a, cf, taps, line_h2n, cs);
    if (e != hipSuccess) return e;
    return launch_pcg(st, 2, pcg_args(pt, ugrid_ez(N), P, cf, part, pst, rtol), max_iter, ez,
                      tracked ? ge : nullptr, t1, cf);
}

hipError_t launch_pcg_h_2d(hipStream_t st, bool tracked, const double* src, double* hx, double* hy, double* t1,
                           int N, int P, const Coef& cf, const PadeTaps& taps, const PadeLine& line_n2h,
                           const ChebSchedule& cs, double* const* pt, double* part, PcgState* pst, double rtol,
                           int max_iter)
{
    ColArgs ax{src, nullptr, nullptr, hx, nullptr, ugrid_hx(N), N, P, pt[1], nullptr};
    hipError_t e = tracked ? launch_col_rhs<COL_HX_TRACKED>(st, ax, cf, taps, line_n2h, cs)
                           : launch_col_rhs<COL_HX_DISCRETE>(st, ax, cf, taps, line_n2h, cs);
    if (e != hipSuccess) return e;
    e = launch_pcg(st, 2, pcg_args(pt, ugrid_hx(N), P, cf, part, pst, rtol), max_iter, hx, nullptr, nullptr, cf);
    if (e != hipSuccess) return e;
    // Hy: the x-line right-hand side T1 is b
    double* pty[7] = {pt[0], t1, pt[2], pt[3], pt[4], pt[5], pt[6]};
    return launch_pcg(st, 2, pcg_args(pty, ugrid_hy(N), P, cf, part, pst, rtol), max_iter, hy, nullptr, nullptr,
                      cf);
}

// The same right-hand sides as the PCG form, solved by the transforms
// (pt[0], pt[2]: work arrays; pt[1]: b).
hipError_t launch_tsolve_e_2d(hipStream_t st, bool tracked, const double* hx, double* ez, double* ge,
                              const double* t0, double* t1, int N, int P, const Coef& cf, const PadeTaps& taps,
                              const PadeLine& line_h2n, const ChebSchedule& cs, double* const* pt,
                              const TransformTables& tt)
{
    ColArgs a{hx, t0, t1, ez, ge, ugrid_ez(N), N, P, pt[1], t1};
    hipError_t e = tracked ? launch_col_rhs<COL_E_TRACKED>(st, a, cf, taps, line_h2n, cs)
                           : launch_col_rhs<COL_E_DISCRETE>(st, a, cf, taps, line_h2n, cs);
    if (e != hipSuccess) return e;
    return launch_transform_solve(st, 2, tt, ugrid_ez(N), P, 0, pt[1], pt[0], pt[2], ez, tracked ? ge : nullptr, t1,
                                  cf);
}

hipError_t launch_tsolve_h_2d(hipStream_t st, bool tracked, const double* src, double* hx, double* hy, double* t1,
                              int N, int P, const Coef& cf, const PadeTaps& taps, const PadeLine& line_n2h,
                              const ChebSchedule& cs, double* const* pt, const TransformTables& tt)
{
    ColArgs ax{src, nullptr, nullptr, hx, nullptr, ugrid_hx(N), N, P, pt[1], nullptr};
    hipError_t e = tracked ? launch_col_rhs<COL_HX_TRACKED>(st, ax, cf, taps, line_n2h, cs)
                           : launch_col_rhs<COL_HX_DISCRETE>(st, ax, cf, taps, line_n2h, cs);
    if (e != hipSuccess) return e;
    e = launch_transform_solve(st, 2, tt, ugrid_hx(N), P, 0, pt[1], pt[0], pt[2], hx, nullptr, nullptr, cf);
    if (e != hipSuccess) return e;
    // Hy: the x-line right-hand side T1 is b
    return launch_transform_solve(st, 2, tt, ugrid_hy(N), P, 0, t1, pt[0], pt[2], hy, nullptr, nullptr, cf);
}

}  // namespace c4m
