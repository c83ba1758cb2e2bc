// c4m_stream_2d.h -- streaming form of the 2D column kernel (FP64 solve).
//
// One wavefront owns a strip of 64 adjacent columns and a segment of OH
// output rows and walks down the segment one row per step, with no LDS and
// no barriers:
//   * the y-line Pade derivative (Section 3.4, Appendix A.1) of the streamed
//     source comes from a 28-row register window (truncated A^{-1} D, exact
//     rows near the line ends from the table);
//   * the right-hand side b of the row is formed from it, the part across
//     the line of the source conditioning G (a second difference between
//     neighbouring columns) and the precomputed x-line part;
//   * the K Chebyshev applications of M = alpha I - beta L9 run as a
//     pipeline: application k works on the row k rows above the newest b
//     row, so it sees the rows above and below it from the previous
//     application; the 9-point column sums cross between columns through
//     DPP lane shifts;
//   * the row that leaves the last application is the solve's result and
//     updates the field (and G_E) at once.
// A region of OH + 2K rows and 64 columns gives exact results on its OH
// inner rows and 64 - 2 (K + 1) inner columns (K for the solve, one more
// for the cross-line part of G), as in the tile form.
#pragma once
#include "c4m_tiles_2d.h"

namespace c4m {

// Value held by lane l - 1 (by lane l + 1), 0 in lane 0 (lane 63): DPP
// wavefront shifts by one lane, each half of the double separately.
__device__ __forceinline__ double from_left(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_right(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

constexpr int SW_COLS = 64;          // columns of a strip (one wavefront)
constexpr int SW_WIN = COND_TAPS;    // raw rows in the Pade window
constexpr int SW_WAVES = 4;          // strips per workgroup

// Strip shapes: TRX region rows (OH = TRX - 2 K output rows), unrolled U
// steps at a time, per-row inputs fetched LA steps ahead.
template <int K, int MODE, int TRX, int U, int LA>
struct StripShape {
    static constexpr int OH = TRX - 2 * K;
    static constexpr bool YPART = MODE != COL_HY;
    static constexpr bool SPLIT = MODE == COL_E_TRACKED || MODE == COL_E_DISCRETE || MODE == COL_HX_DISCRETE;
    static constexpr bool ESTEP = MODE == COL_E_TRACKED || MODE == COL_E_DISCRETE;
    static constexpr bool HAS_T0 = ESTEP || MODE == COL_HY;
    static constexpr bool CARRY = MODE == COL_E_TRACKED;
    static constexpr int HX = K + (SPLIT ? 1 : 0);   // halo columns on each side
    static constexpr int OW = SW_COLS - 2 * HX;     // output columns
    static constexpr int TR = TRX;                  // region rows = steps
    static constexpr int NW = YPART ? SW_WIN + LA : 1;
    static constexpr int NQ = LA + 1;               // per-row prefetch queue
    static_assert(TR % U == 0, "region rows must be a multiple of the unroll");
    static_assert(OW > 0 && OH > 0, "strip too small for K");
};

template <class SS>
__host__ __device__ inline int strip_tiles_x(const UGrid& g)
{
    return (g.hi[0] - g.lo[0] + SS::OW - 1) / SS::OW;
}
template <class SS>
__host__ __device__ inline int strip_tiles_y(const UGrid& g)
{
    return (g.hi[1] - g.lo[1] + SS::OH - 1) / SS::OH;
}

// One strip: region columns gx = x0 - HX + lane, output rows [y0, y0 + OH).
// INNER: every region row and column is strictly inside the unknowns and
// every Pade row of the region is an interior row, so no masks and the
// antisymmetric interior taps (pair form) apply.
template <int K, int MODE, int TRX, int U, int LA, bool INNER>
__device__ __forceinline__ void strip_run(const ColArgs& a, const Coef& cf, const PadeLine& L,
                                          const ChebSchedule& cs, int x0, int y0)
{
    using SS = StripShape<K, MODE, TRX, U, LA>;
    constexpr bool YPART = SS::YPART, SPLIT = SS::SPLIT, HAS_T0 = SS::HAS_T0, CARRY = SS::CARRY;
    constexpr int HX = SS::HX, TR = SS::TR, NW = SS::NW, NQ = SS::NQ;
    const int lane = (int)(threadIdx.x % SW_COLS);
    const UGrid& g = a.g;
    const int P = a.P;
    const int gx = x0 - HX + lane;
    const bool col_active = gx >= g.lo[0] && gx < g.hi[0];
    const bool col_data = gx >= 0 && gx <= a.N;
    const bool nx = g.neumann[0], ny = g.neumann[1];
    const bool mlo = nx && gx == g.lo[0], mhi = nx && gx == g.hi[0] - 1;
    const bool lane_out = lane >= HX && lane < SW_COLS - HX && col_active;
    const int ylo = g.lo[1], yhi = g.hi[1];
    const int ry0 = y0 - K;                             // grid row of region row 0
    const int mofs = SS::ESTEP ? 1 : 0;                 // grid row = Pade output index + mofs
    const int mbase = ry0 - mofs;                       // Pade output index of region row 0
    const int gbase = mbase - (SW_WIN / 2 - 1);         // raw row in window slot 0 at region row 0
    const int n_in = L.n_in, n_out = L.n_out;
    const double* __restrict__ src = a.src;
    const double* __restrict__ t0 = a.t0;
    const double* __restrict__ t1 = a.t1;
    double* __restrict__ field = a.field;
    double* __restrict__ ge = a.ge;
    const size_t cofs = (size_t)(col_data ? gx : 0);

    const double b6 = cf.beta * (1.0 / 6.0);
    const double a36 = fma(36.0, b6, cf.alpha);
    const double ysign = SS::ESTEP ? -cf.z : (MODE == COL_HY ? 0.0 : -1.0 / cf.z);

    auto load_raw = [&](int gg) -> double {
        if (INNER) return src[(size_t)gg * P + cofs];
        return (gg >= 0 && gg < n_in && col_data) ? src[(size_t)gg * P + cofs] : 0.0;
    };
    // grid rows of the per-row inputs: t0 of region row ry; field, G_E and
    // t1 of the output row that leaves the pipeline at step ry
    auto row_act = [&](int gy) -> bool { return INNER ? true : (col_active && gy >= ylo && gy < yhi); };
    auto load_t0 = [&](int ry) -> double {
        const int gy = ry0 + ry;
        return (ry < TR && row_act(gy)) ? t0[(size_t)gy * P + cofs] : 0.0;
    };
    auto out_row = [&](int ry) -> bool {   // step ry updates grid row ry0 + ry - K
        const int gy = ry0 + ry - K;
        return ry >= 2 * K && ry < TR && gy < yhi;
    };

    // ---- state
    double fw[NW];                 // raw window: slot i holds raw row gbase + ry + i
    double t0q[NQ], fq[NQ], gq[NQ], t1q[NQ];
    double pd[K + 1];              // raw Pade derivative of the last K + 1 rows
    double dp1[K], dp2[K], rp1[K], xp1[K];
#pragma unroll
    for (int j = 0; j < K; ++j) dp1[j] = dp2[j] = rp1[j] = xp1[j] = 0.0;
#pragma unroll
    for (int j = 0; j <= K; ++j) pd[j] = 0.0;
    if (YPART) {
#pragma unroll
        for (int i = 1; i < NW; ++i) fw[i] = load_raw(gbase - 1 + i);
    }
#pragma unroll
    for (int i = 1; i < NQ; ++i) {
        const int ry = i - 1;
        t0q[i] = HAS_T0 ? load_t0(ry) : 0.0;
        const bool o = out_row(ry) && lane_out;
        const size_t off = (size_t)(o ? ry0 + ry - K : 0) * P + cofs;
        fq[i] = o ? field[off] : 0.0;
        gq[i] = (CARRY && o) ? ge[off] : 0.0;
        t1q[i] = (CARRY && o) ? t1[off] : 0.0;
    }

    CDouble* tab = as_const(L.rows);
    CDouble* ctab = as_const(L.crows);
    CDouble* pq = as_const(L.pairs);                    // 14 conditioned, then 13 raw pair taps

    for (int blk = 0; blk < TR; blk += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int ry = blk + u;
            // ---- advance the window and the prefetch queues
            if (YPART) {
#pragma unroll
                for (int i = 0; i < NW - 1; ++i) fw[i] = fw[i + 1];
                fw[NW - 1] = load_raw(gbase + ry + NW - 1);
            }
#pragma unroll
            for (int i = 0; i < NQ - 1; ++i) {
                t0q[i] = t0q[i + 1];
                fq[i] = fq[i + 1];
                gq[i] = gq[i + 1];
                t1q[i] = t1q[i + 1];
            }
            {
                const int rn = ry + LA;
                t0q[NQ - 1] = HAS_T0 ? load_t0(rn) : 0.0;
                const bool o = out_row(rn) && lane_out;
                const size_t off = (size_t)(o ? ry0 + rn - K : 0) * P + cofs;
                fq[NQ - 1] = o ? field[off] : 0.0;
                gq[NQ - 1] = (CARRY && o) ? ge[off] : 0.0;
                t1q[NQ - 1] = (CARRY && o) ? t1[off] : 0.0;
            }

            // ---- line derivatives of Pade row m = mbase + ry: raw (pr) and of
            // the conditioned source (cr); the window holds rows m - 13 .. m + 14
            double pr = 0.0, cr = 0.0;
            if (YPART) {
                if (INNER) {
                    double dl[SW_WIN / 2];
#pragma unroll
                    for (int j = 0; j < SW_WIN / 2; ++j) dl[j] = fw[SW_WIN / 2 - 1 - j] - fw[SW_WIN / 2 + j];
#pragma unroll
                    for (int j = 0; j < PADE_TAPS / 2; ++j) pr = fma(pq[SW_WIN / 2 + j], dl[j], pr);
                    if (SPLIT) {
#pragma unroll
                        for (int j = 0; j < SW_WIN / 2; ++j) cr = fma(pq[j], dl[j], cr);
                    } else {
                        cr = pr;
                    }
                } else {
                    const int m = mbase + ry;
                    if (m >= 0 && m < n_out) {
                        const int row = pade_row_index(L, m);
                        CDouble* tp = tab + (size_t)row * PADE_TAPS;
#pragma unroll
                        for (int u2 = 0; u2 < PADE_TAPS; ++u2) pr = fma(tp[u2], fw[1 + u2], pr);
                        if (SPLIT) {
                            CDouble* tq = ctab + (size_t)row * COND_TAPS;
#pragma unroll
                            for (int w = 0; w < COND_TAPS; ++w) cr = fma(tq[w], fw[w], cr);
                        } else {
                            cr = pr;
                        }
                    }
                }
            }

            // ---- right-hand side of region row ry
            const int gy = ry0 + ry;
            double b = 0.0;
            {
                double v = 0.0;
                if (YPART) {
                    double s = cr;
                    if (SPLIT) s += (from_left(pr) + from_right(pr) - 2.0 * pr) * (1.0 / 12.0);
                    v = ysign * s;
                }
                if (HAS_T0) v += t0q[0];
                b = row_act(gy) ? v : 0.0;
            }
            if (CARRY) {
#pragma unroll
                for (int j = 0; j < K; ++j) pd[j] = pd[j + 1];
                pd[K] = pr;
            }

            // ---- Chebyshev pipeline: application j + 1 on row ry - j - 1
            double dn[K + 1], rn[K + 1], xn[K + 1];
            dn[0] = b * cs.inv_theta;
            rn[0] = b;
            xn[0] = 0.0;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int gq_ = gy - j - 1;
                double up = dp2[j], cen = dp1[j], dw = dn[j];
                if (!INNER) {
                    if (ny && gq_ == ylo) up = cen;
                    if (ny && gq_ == yhi - 1) dw = cen;
                }
                const double sown = fma(4.0, cen, up + dw);
                double sl = from_left(sown), sr = from_right(sown);
                if (!INNER) {
                    if (mlo) sl = sown;
                    if (mhi) sr = sown;
                }
                const double ad = fma(a36, cen, -b6 * fma(4.0, sown, sl + sr));
                xn[j + 1] = j == 0 ? cen : xp1[j] + cen;
                double r_ = rp1[j] - ad;
                double d_ = fma(cs.c1[j], cen, cs.c2[j] * r_);
                if (!INNER) {
                    const bool act = col_active && gq_ >= ylo && gq_ < yhi;
                    r_ = act ? r_ : 0.0;
                    d_ = act ? d_ : 0.0;
                }
                rn[j + 1] = r_;
                dn[j + 1] = d_;
            }
#pragma unroll
            for (int j = 0; j < K; ++j) {
                dp2[j] = dp1[j];
                dp1[j] = dn[j];
                rp1[j] = rn[j];
                xp1[j] = xn[j];
            }

            // ---- update of grid row gy - K
            if (out_row(ry) && lane_out) {
                const double phi = xn[K] + dn[K];
                const size_t o = (size_t)(gy - K) * P + cofs;
                const double de = cf.cfl * phi;
                field[o] = fq[0] + de;
                if (CARRY) ge[o] = gq[0] + fma(cf.ge_gain, de, -cf.ge_curl * (t1q[0] - pd[0]));
            }
        }
    }
}

template <int K, int MODE, int TRX, int U, int LA>
__device__ __forceinline__ void strip_tile(const ColArgs& a, const Coef& cf, const PadeLine& L,
                                           const ChebSchedule& cs, int bxi, int byi)
{
    using SS = StripShape<K, MODE, TRX, U, LA>;
    const UGrid& g = a.g;
    const int x0 = g.lo[0] + bxi * SS::OW;
    const int y0 = g.lo[1] + byi * SS::OH;
    const int rx0 = x0 - SS::HX, ry0 = y0 - K;
    const int mofs = SS::ESTEP ? 1 : 0;
    bool inner = rx0 > g.lo[0] && rx0 + SW_COLS < g.hi[0] && ry0 > g.lo[1] && ry0 + SS::TR < g.hi[1];
    if (SS::YPART) {
        // Pade rows of the region are interior rows; the window rows stay in the line
        const int m_lo = ry0 - mofs, m_hi = ry0 - mofs + SS::TR - 1;
        inner = inner && pade_interior(L, m_lo, m_hi) && m_lo - SW_WIN / 2 >= 0 &&
                m_hi + SW_WIN / 2 + SS::NW - SW_WIN < L.n_in;
    }
    if (inner)
        strip_run<K, MODE, TRX, U, LA, true>(a, cf, L, cs, x0, y0);
    else
        strip_run<K, MODE, TRX, U, LA, false>(a, cf, L, cs, x0, y0);
}

}  // namespace c4m
