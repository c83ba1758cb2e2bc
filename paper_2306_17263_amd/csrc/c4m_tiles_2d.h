// c4m_tiles_2d.h -- 2D TM (Ez, Hx, Hy) tile code shared by the
// single-problem launches (c4m_kernels_2d.hip) and the batched form
// (c4m_batch.hip): the x-line tiles of both steps and the column-tile form
// of the solve.  The default single-problem solve, the wave strips, is in
// c4m_stream_2d.h.
//
// Step 1 (Section 3.4): the x-lines of Hy give the x part of the right-hand
// side (T0 = Z delta_x G(Hy), or only the raw derivative P = delta_x Hy,
// from which the strips form T0); the solve kernel adds the y-line part
// -Z delta_y G(Hx), solves M Phi = b and updates Ez += r Phi and
// G_E += (1 + 4/r^2) r Phi - (2/r) Z curl^A H.
// Step 2: the x-lines of G_E give T1 = (1/Z) delta_x G_E (the Hy
// right-hand side); the Hx solve forms -(1/Z) delta_y G_E itself.
// G_E = alpha E + l/12 is stored instead of l, so Step 2 reads only G_E.
//
// Pade derivative: A^{-1} D truncated to 2 PADE_R + 2 taps on the line
// values (exact rows near the two ends of each line from a table).
// Source conditioning G u = alpha u + (L5 u)/12 is split by axis: the part
// along the line is folded into the line input, the part across the line is
// applied to the line derivatives of the neighbouring lines (the line
// derivative is the same linear map on every line, so the two commute).
//
// Column tiles (k_col): a workgroup holds a region of 128 (or 64) columns;
// NL lanes per column keep its region rows in registers; the column sums
// S = d(y-1) + 4 d(y) + d(y+1) of the 9-point stencil cross lanes in LDS.
#pragma once
#include "c4m_internal.h"

namespace c4m {

// Read-only device memory seen through the AMDGPU constant address space
// (loads with a wave-uniform address become scalar loads).
typedef const __attribute__((address_space(4))) double CDouble;
__device__ __forceinline__ CDouble* as_const(const double* p)
{
    return (CDouble*)p;
}

// table row of Pade output m: explicit rows near the ends, else the
// interior row stored after them
__host__ __device__ inline int pade_row_index(const PadeLine& L, int m)
{
    if (L.all || m < L.b) return m;
    if (m >= L.n_out - L.b) return m - (L.n_out - L.b) + L.b;
    return 2 * L.b;
}

__device__ __forceinline__ const double* pade_row(const PadeLine& L, int m)
{
    return L.rows + (size_t)pade_row_index(L, m) * PADE_TAPS;
}

__device__ __forceinline__ bool pade_interior(const PadeLine& L, int m_lo, int m_hi)
{
    // every output in [m_lo, m_hi] uses the interior taps
    return !L.all && m_lo >= L.b && m_hi < L.n_out - L.b;
}

// ===========================================================================
// x-lines.  Tile: 32 rows x 64 outputs, 256 threads; thread (row = t % 32,
// seg = t / 32) computes 8 consecutive outputs from a 33-value register
// window.  Lanes 0..15 and 16..31 of a wave read 16 consecutive rows at the
// same column, and the odd LDS row stride keeps those reads conflict-free.
// ===========================================================================
constexpr int XT_ROWS = 32;
constexpr int XT_OUT = 64;
constexpr int XT_SEG = 8;
constexpr int XT_IN = XT_OUT + 2 * PADE_R + 2;     // staged inputs per row
constexpr int XT_STRIDE = XT_IN + 1;               // odd
constexpr int XT_WIN = XT_SEG + PADE_TAPS - 1;

enum { XL_E_TRACKED = 0, XL_E_DISCRETE = 1, XL_H_TRACKED = 2, XL_H_DISCRETE = 3 };

struct XArgs {
    const double* src;      // Hy (Step 1) or G_E / Ez (Step 2)
    double* t0;
    double* t1;
    int N, P;
    PadeLine L;
};

// LDS doubles the x-line tiles take from the caller's buffer (the raw
// line input as well in the Step 1 mode with the carried Laplacian)
constexpr int xt_lds(int mode) { return (mode == XL_E_TRACKED ? 2 : 1) * XT_ROWS * XT_STRIDE; }

template <int MODE>
__device__ __forceinline__ void xlines_tile(const double* __restrict__ src, double* __restrict__ t0,
                                            double* __restrict__ t1, int N, int P, const PadeLine& L,
                                            const Coef& cf, const PadeTaps& taps, int bxi, int byi,
                                            double* lds)
{
    constexpr bool E = MODE == XL_E_TRACKED || MODE == XL_E_DISCRETE;
    constexpr bool TWO = MODE == XL_E_TRACKED;     // raw derivative as well
    double* sg = lds;                               // [XT_ROWS * XT_STRIDE]
    double* sr = lds + XT_ROWS * XT_STRIDE;         // (TWO)
    const int tid = threadIdx.x;
    const int m0 = bxi * XT_OUT;                    // first output of the tile
    const int j0 = 1 + byi * XT_ROWS;               // first row (interior rows 1..N-1)
    const int n_in = L.n_in;
    // ---- stage the conditioned line input (and the raw one).  Chunks of CH
    // elements per thread: the loads of a chunk take clamped (valid)
    // addresses and are all issued before its LDS stores.
    constexpr int NS = (XT_ROWS * XT_IN + 255) / 256;
    constexpr int CH = MODE == XL_H_TRACKED ? NS : 4;
    for (int i0 = 0; i0 < NS; i0 += CH) {
        double vg[CH], vr[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int e = tid + (i0 + c) * 256;
            const int rr = e / XT_IN, q = e - rr * XT_IN;
            const int j = j0 + rr, g = m0 - PADE_R + q;
            const bool ok = i0 + c < NS && e < XT_ROWS * XT_IN && j <= N - 1 && g >= 0 && g < n_in;
            const int jc = ok ? j : 1, gc = ok ? g : 0;
            const double* row = src + (size_t)jc * P;
            double a = 0.0, b = 0.0;
            if (E) {
                // Hy at half points along x: even ghosts at both ends
                const double h0 = row[gc];
                const double hl = row[gc > 0 ? gc - 1 : 0];
                const double hr = row[gc < n_in - 1 ? gc + 1 : n_in - 1];
                const double hs = row[gc - P];
                const double hn = row[gc + P];
                b = h0;
                a = fma(cf.alpha, h0, (hl + hr + hs + hn - 4.0 * h0) * (1.0 / 12.0));
            } else if (MODE == XL_H_TRACKED) {
                a = row[gc];                                       // stored G_E
            } else {
                // alpha E + L5 E / 12, zero on the walls (nodes 0 and N)
                const int gi = gc < 1 ? 1 : (gc > n_in - 2 ? n_in - 2 : gc);
                const double e0 = row[gi];
                const double w = fma(cf.alpha, e0, (row[gi - 1] + row[gi + 1] + row[gi - P] + row[gi + P] - 4.0 * e0) *
                                                       (1.0 / 12.0));
                a = (gc > 0 && gc < n_in - 1) ? w : 0.0;
            }
            vg[c] = ok ? a : 0.0;
            vr[c] = ok ? b : 0.0;
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int e = tid + (i0 + c) * 256;
            const int rr = e / XT_IN, q = e - rr * XT_IN;
            if (i0 + c < NS && e < XT_ROWS * XT_IN) {
                sg[rr * XT_STRIDE + q] = vg[c];
                if (TWO) sr[rr * XT_STRIDE + q] = vr[c];
            }
        }
    }
    __syncthreads();
    const int row = tid % XT_ROWS;
    const int seg = tid / XT_ROWS;
    const int mb = m0 + seg * XT_SEG;
    double outg[XT_SEG], outr[XT_SEG];
    const double* wg = sg + row * XT_STRIDE + seg * XT_SEG;
    const double* wr = sr + row * XT_STRIDE + seg * XT_SEG;
    if (pade_interior(L, mb, mb + XT_SEG - 1)) {
        double w[XT_WIN];
#pragma unroll
        for (int u = 0; u < XT_WIN; ++u) w[u] = wg[u];
#pragma unroll
        for (int k = 0; k < XT_SEG; ++k) {
            double a = 0.0;
#pragma unroll
            for (int u = 0; u < PADE_TAPS; ++u) a = fma(taps.c[u], w[k + u], a);
            outg[k] = a;
        }
        if (TWO) {
#pragma unroll
            for (int u = 0; u < XT_WIN; ++u) w[u] = wr[u];
#pragma unroll
            for (int k = 0; k < XT_SEG; ++k) {
                double a = 0.0;
#pragma unroll
                for (int u = 0; u < PADE_TAPS; ++u) a = fma(taps.c[u], w[k + u], a);
                outr[k] = a;
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < XT_SEG; ++k) {
            const int m = mb + k;
            double a = 0.0, b = 0.0;
            if (m < L.n_out) {
                const double* cr = pade_row(L, m);
                for (int u = 0; u < PADE_TAPS; ++u) {
                    const double c = cr[u];
                    a = fma(c, wg[k + u], a);
                    if (TWO) b = fma(c, wr[k + u], b);
                }
            }
            outg[k] = a;
            outr[k] = b;
        }
    }
    // ---- write through the LDS so that a wave stores contiguous row segments:
    // E step -> node i = m + 1; H step -> half point i = m
    __syncthreads();
    constexpr int OS = XT_OUT + 1;
    double* og = sg;                        // [XT_ROWS][OS], reuses the staging area
    double* orw = TWO ? sr : sg;
#pragma unroll
    for (int k = 0; k < XT_SEG; ++k) {
        og[row * OS + seg * XT_SEG + k] = outg[k];
        if (TWO) orw[row * OS + seg * XT_SEG + k] = outr[k];
    }
    __syncthreads();
    const int ioff = E ? 1 : 0;
    const double scale = E ? cf.z : 1.0 / cf.z;
    double* o0 = E ? t0 : t1;
    for (int e = tid; e < XT_ROWS * XT_OUT; e += 256) {
        const int rr = e / XT_OUT, c = e - rr * XT_OUT;
        const int jj = j0 + rr, m = m0 + c;
        if (jj <= N - 1 && m < L.n_out) {
            o0[(size_t)jj * P + m + ioff] = scale * og[rr * OS + c];
            if (TWO) t1[(size_t)jj * P + m + ioff] = orw[rr * OS + c];
        }
    }
}

// ===========================================================================
// x-lines of Step 1 from raw derivatives only.  The conditioning G splits
// into the part along the line and the part across it; the derivative
// along the line commutes with both away from the line ends (interior
// Toeplitz rows), so with P = the raw line derivative of a row
//   T0 = Z (alpha P + (P(m-1) + P(m+1) - 2 P(m)) / 12 + (P_s + P_n - 2 P) / 12)
// (P_s, P_n: the rows below and above), and T1 = P.  Near the line ends
// the along-line part comes from the conditioned table rows instead.
// Tile: P on 32 rows (j0 - 1 .. j0 + 30) x 64 outputs (m0 - 1 .. m0 + 62),
// 256 threads, 8 outputs per thread from a register window; T0 and T1 on
// the inner 30 x 62.
// ===========================================================================
constexpr int XE_PROWS = 32;
constexpr int XE_OROWS = XE_PROWS - 2;
constexpr int XE_POUT = 64;
constexpr int XE_OUT = XE_POUT - 2;
constexpr int XE_SEG = 8;
constexpr int XE_IN = XE_POUT + PADE_TAPS - 1;     // staged inputs per row (89)
constexpr int XE_STRIDE = XE_IN + 2;               // odd
constexpr int XE_PSTRIDE = XE_POUT + 1;            // odd
constexpr int XE_WIN = XE_SEG + PADE_TAPS - 1;

__host__ __device__ inline int xe_tiles_x(int n_out) { return (n_out + XE_OUT - 1) / XE_OUT; }
__host__ __device__ inline int xe_tiles_y(int N) { return (N - 1 + XE_OROWS - 1) / XE_OROWS; }

// PF (strip form): the tile writes P itself to t1 on rows 0..N (the strips
// form T0 from it) and T0 only on the band columns of the line ends (where
// the along-line part needs the conditioned table rows) to t0.
constexpr int XE_LDS = XE_PROWS * XE_STRIDE + XE_PROWS * XE_PSTRIDE;

template <bool TWO, bool PF>
__device__ __forceinline__ void xlines_e_tile(const double* __restrict__ src, double* __restrict__ t0,
                                              double* __restrict__ t1, int N, int P, const PadeLine& L,
                                              const Coef& cf, int bxi, int byi, double* lds)
{
    double* sh = lds;                                  // raw rows, later the T0 tile
    double* sp = lds + XE_PROWS * XE_STRIDE;           // P
    const int tid = threadIdx.x;
    const int m0 = bxi * XE_OUT;                       // first T0 output of the tile
    const int j0 = 1 + byi * XE_OROWS;                 // first T0 row
    const int n_in = L.n_in, n_out = L.n_out;
    const int g0 = m0 - 1 - PADE_R;                    // line position of staged column 0
    // ---- stage the raw rows j0 - 1 .. j0 + 30 (zero off the grid and line).
    // Every load of the thread is issued before the first LDS store: the
    // loads take clamped (valid) addresses and the value is selected after.
    {
        constexpr int NS = (XE_PROWS * XE_IN + 255) / 256;
        double v[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            const int e = tid + i * 256;
            const int rr = e / XE_IN, q = e - rr * XE_IN;
            const int j = j0 - 1 + rr, g = g0 + q;
            const bool ok = e < XE_PROWS * XE_IN && j <= N && g >= 0 && g < n_in;
            const double x = src[ok ? (size_t)j * P + g : 0];
            v[i] = ok ? x : 0.0;
        }
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            const int e = tid + i * 256;
            const int rr = e / XE_IN, q = e - rr * XE_IN;
            if (e < XE_PROWS * XE_IN) sh[rr * XE_STRIDE + q] = v[i];
        }
    }
    __syncthreads();
    // ---- P on the 32 x 64 outputs; 8 per thread
    const int row = tid % XE_PROWS;
    const int seg = tid / XE_PROWS;
    const int mb = m0 - 1 + seg * XE_SEG;              // Pade output of this thread's first P
    const double* w = sh + row * XE_STRIDE + seg * XE_SEG;   // staged position of f[mb - 12]
    double pv[XE_SEG];
    const bool fast = pade_interior(L, mb, mb + XE_SEG - 1);
    if (fast) {
        CDouble* tc = as_const(L.rows + (size_t)(2 * L.b) * PADE_TAPS);
        double f[XE_WIN];
#pragma unroll
        for (int u = 0; u < XE_WIN; ++u) f[u] = w[u];
#pragma unroll
        for (int k = 0; k < XE_SEG; ++k) pv[k] = 0.0;
#pragma unroll
        for (int u = 0; u < PADE_TAPS; ++u) {
            const double c = tc[u];
#pragma unroll
            for (int k = 0; k < XE_SEG; ++k) pv[k] = fma(c, f[k + u], pv[k]);
        }
    } else {
#pragma unroll
        for (int k = 0; k < XE_SEG; ++k) {
            const int m = mb + k;
            double a = 0.0;
            if (m >= 0 && m < n_out) {
                CDouble* cr = as_const(pade_row(L, m));
                for (int u = 0; u < PADE_TAPS; ++u) a = fma(cr[u], w[k + u], a);
            }
            pv[k] = a;
        }
    }
#pragma unroll
    for (int k = 0; k < XE_SEG; ++k) sp[row * XE_PSTRIDE + seg * XE_SEG + k] = pv[k];
    __syncthreads();
    if (PF) {
        // P on the inner rows, and on rows 0 and N (first and last tile)
        for (int e = tid; e < XE_PROWS * XE_OUT; e += 256) {
            const int rp = e / XE_OUT, c = e - rp * XE_OUT;
            const int jj = j0 - 1 + rp, m = m0 + c;
            const bool keep = (rp >= 1 && rp <= XE_OROWS && jj <= N - 1) || jj == 0 || jj == N;
            if (keep && jj <= N && m < n_out) t1[(size_t)jj * P + m + 1] = sp[rp * XE_PSTRIDE + c + 1];
        }
        if (!(L.all || m0 <= L.b || m0 + XE_OUT - 1 >= n_out - 1 - L.b)) return;
        // T0 on the band columns: conditioned table rows along the line
        for (int e = tid; e < XE_OROWS * XE_OUT; e += 256) {
            const int rr = e / XE_OUT, c = e - rr * XE_OUT;
            const int jj = j0 + rr, m = m0 + c;
            if (jj > N - 1 || m >= n_out || !(L.all || m <= L.b || m >= n_out - 1 - L.b)) continue;
            const double* q = sp + (rr + 1) * XE_PSTRIDE + c + 1;
            const double pc = q[0];
            const double across = (q[-XE_PSTRIDE] + q[XE_PSTRIDE] - 2.0 * pc) * (1.0 / 12.0);
            CDouble* cr = as_const(L.crows + (size_t)pade_row_index(L, m) * COND_TAPS);
            const double* wr = sh + (rr + 1) * XE_STRIDE + c;   // staged f[m - 13]
            double along = 0.0;
            for (int u = 0; u < COND_TAPS; ++u) along = fma(cr[u], wr[u], along);
            t0[(size_t)jj * P + m + 1] = cf.z * (along + across);
        }
        return;
    }
    // ---- T0 on the inner rows and outputs, through the LDS for row stores
    double t0v[XE_SEG];
    const bool out_row = row >= 1 && row <= XE_OROWS;
#pragma unroll
    for (int k = 0; k < XE_SEG; ++k) {
        const int c = seg * XE_SEG + k;                // P column (output m = mb + k)
        const int m = mb + k;
        double v = 0.0;
        if (out_row && c >= 1 && c <= XE_OUT) {
            const double* q = sp + row * XE_PSTRIDE + c;
            const double pc = q[0];
            const double across = (q[-XE_PSTRIDE] + q[XE_PSTRIDE] - 2.0 * pc) * (1.0 / 12.0);
            double along;
            if (!L.all && m - 1 >= L.b && m + 1 < n_out - L.b) {
                along = fma(cf.alpha, pc, (q[-1] + q[1] - 2.0 * pc) * (1.0 / 12.0));
            } else {
                along = 0.0;
                if (m >= 0 && m < n_out) {
                    // conditioned table row: raw positions m - 13 .. m + 14
                    CDouble* cr = as_const(L.crows + (size_t)pade_row_index(L, m) * COND_TAPS);
                    const double* wr = sh + row * XE_STRIDE + c - 1;   // staged f[m - 13]
                    for (int u = 0; u < COND_TAPS; ++u) along = fma(cr[u], wr[u], along);
                }
            }
            v = cf.z * (along + across);
        }
        t0v[k] = v;
    }
    __syncthreads();
    constexpr int OS = XE_OUT + 1;
    if (out_row) {
#pragma unroll
        for (int k = 0; k < XE_SEG; ++k) {
            const int c = seg * XE_SEG + k;
            if (c >= 1 && c <= XE_OUT) sh[(row - 1) * OS + c - 1] = t0v[k];
        }
    }
    __syncthreads();
    // E step: node i = m + 1
    for (int e = tid; e < XE_OROWS * XE_OUT; e += 256) {
        const int rr = e / XE_OUT, c = e - rr * XE_OUT;
        const int jj = j0 + rr, m = m0 + c;
        if (jj <= N - 1 && m < n_out) {
            t0[(size_t)jj * P + m + 1] = sh[rr * OS + c];
            if (TWO) t1[(size_t)jj * P + m + 1] = sp[(rr + 1) * XE_PSTRIDE + c + 1];
        }
    }
}

// ===========================================================================
// Column kernel: y-line Pade + Chebyshev solve + update.
// A workgroup covers a region of CW = 128 columns and TR rows.  The column
// of region row r is held by NL lanes: lane (c, q) keeps rows
// [q HR, (q+1) HR) of column c in registers.  The rows next to a split
// cross through a small double-buffered LDS array, the column sums
// S = d(y-1) + 4 d(y) + d(y+1) of the 9-point stencil cross between
// columns through the LDS (padded rows, zero sentinels at both ends).
// ===========================================================================
// Column-kernel tile shapes: CW region columns, NL lanes per column.
template <int CW_, int NL_>
struct TileShape {
    static constexpr int CW = CW_;
    static constexpr int CWP = CW_ + 2;      // LDS row stride (zero sentinels at both ends)
    static constexpr int NL = NL_;
    static constexpr int NTC = CW_ * NL_;    // threads per workgroup
};
using Shape0 = TileShape<128, 4>;            // default
using Shape1 = TileShape<64, 4>;
using Shape2 = TileShape<128, 2>;
constexpr int NSHAPES = 3;

// region rows for K sweeps: at least 16 output rows, a multiple of NL
template <int K, class S>
struct ColShape {
    static constexpr int TR = ((16 + 2 * K + S::NL - 1) / S::NL) * S::NL;
    static constexpr int OH = TR - 2 * K;
    static constexpr int HR = TR / S::NL;
};

enum { COL_E_TRACKED = 0, COL_E_DISCRETE = 1, COL_HX_TRACKED = 2, COL_HX_DISCRETE = 3, COL_HY = 4 };

// What the column tile does after forming the right-hand side: the FP64
// Chebyshev solve and update, the FP32-refined solve and update, or only
// store the right-hand side (and the raw curl for the G_E update) for a
// separate solver.
enum { FORM_FP64 = 0, FORM_MIXED = 1, FORM_RHS = 2 };

struct ColArgs {
    const double* src;      // y-line source: Hx (E step) or G_E / Ez (Hx step)
    const double* t0;       // precomputed right-hand side part (T0 or T1), or null
    const double* t1;       // carried Laplacian: x part of curl^A H (E step)
    double* field;          // Ez, Hx or Hy
    double* ge;             // G_E (E step, carried Laplacian)
    UGrid g;                // unknowns of the solved component
    int N, P;
    double* b_out;          // FORM_RHS: right-hand side on the unknowns
    double* cv_out;         // FORM_RHS, carried Laplacian: curl^A H (may alias t1)
    double* yb = nullptr;   // strip form: y-line derivatives near the line ends
};

// Per-lane boundary description of a column tile; the row masks are
// recomputed where needed rather than held in registers.
struct ColCtx {
    bool inner;                     // region strictly inside the unknowns: no boundary handling
    bool mirror_lo_x, mirror_hi_x;  // Neumann mirror of the column sums at the x ends
    bool col_active, ny;            // the column holds unknowns; Neumann along y
    int gy0, ylo, yhi;              // grid row of this lane's row 0; unknown rows [ylo, yhi)
    int part, lane;
    __device__ __forceinline__ bool act(int t) const
    {
        const int gy = gy0 + t;
        return col_active && gy >= ylo && gy < yhi;
    }
};

// (M v)[t] on this lane's rows, handed to upd(t, m, act) row by row (m is
// zero off the unknowns), with L9 v = (S(x-1) + S(x+1) + 4 S(x) - 36 v) / 6
// and S = v(y-1) + 4 v(y) + v(y+1).  The rows next to the part split cross
// through bnd; the column sums through the LDS.  upd may overwrite v[t]:
// row t is the last use of v[t].  Two barriers; inner tiles take a path
// without boundary tests.
template <int HR, class S, class T, class F>
__device__ __forceinline__ void apply_m(const ColCtx& c, const T (&v)[HR], T* lds, T* bnd, double alpha,
                                        double beta, F&& upd)
{
    constexpr int CW = S::CW, CWP = S::CWP, NL = S::NL;
    bnd[(c.part * 2 + 0) * CW + c.lane] = v[0];   // [part][first/last][column]
    bnd[(c.part * 2 + 1) * CW + c.lane] = v[HR - 1];
    __syncthreads();
    const T above = c.part > 0 ? bnd[((c.part - 1) * 2 + 1) * CW + c.lane] : T(0);
    const T below = c.part < NL - 1 ? bnd[((c.part + 1) * 2 + 0) * CW + c.lane] : T(0);
    T* my = lds + c.lane + 1 + c.part * HR * CWP;
    const T b6 = T(beta * (1.0 / 6.0));
    const T a36 = T(fma(36.0, beta * (1.0 / 6.0), alpha));
    T sown[HR];
    if (c.inner) {
#pragma unroll
        for (int t = 0; t < HR; ++t) {
            const T up = t > 0 ? v[t - 1] : above;
            const T dn = t < HR - 1 ? v[t + 1] : below;
            sown[t] = fma(T(4), v[t], up + dn);
            my[t * CWP] = sown[t];
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < HR; ++t) {
            const T* q = my + t * CWP;
            upd(t, fma(a36, v[t], -b6 * fma(T(4), sown[t], q[-1] + q[1])), true);
        }
    } else {
#pragma unroll
        for (int t = 0; t < HR; ++t) {
            const int gy = c.gy0 + t;
            T up = t > 0 ? v[t - 1] : above;
            T dn = t < HR - 1 ? v[t + 1] : below;
            if (c.ny && gy == c.ylo) up = v[t];
            if (c.ny && gy == c.yhi - 1) dn = v[t];
            sown[t] = fma(T(4), v[t], up + dn);
            my[t * CWP] = sown[t];
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < HR; ++t) {
            const T* q = my + t * CWP;
            T sl = q[-1], sr = q[1];
            if (c.mirror_lo_x) sl = sown[t];
            if (c.mirror_hi_x) sr = sown[t];
            const T m = fma(a36, v[t], -b6 * fma(T(4), sown[t], sl + sr));
            const bool a = c.act(t);
            upd(t, a ? m : T(0), a);
        }
    }
}

// One FP32 Chebyshev round of NSW applications of M on the FP64 right-hand
// side b (unchanged); x receives the round's solution.
template <int HR, class S, int NSW>
__device__ __forceinline__ void cheb32(const ColCtx& c, const double (&b)[HR], float (&x)[HR], float* lds,
                                       float* bnd, const Coef& cf, const ChebSchedule& cs)
{
    float d[HR], r[HR];
#pragma unroll
    for (int t = 0; t < HR; ++t) {
        r[t] = (float)b[t];
        d[t] = r[t] * cs.inv_thetaf;
        x[t] = 0.f;
    }
#pragma unroll
    for (int k = 0; k < NSW; ++k) {
        const float c1 = cs.c1f[k], c2 = cs.c2f[k];
        apply_m<HR, S>(c, d, lds, bnd, cf.alpha, cf.beta, [&](int t, float m, bool a) {
            x[t] += d[t];
            r[t] -= m;
            d[t] = a ? fmaf(c1, d[t], c2 * r[t]) : 0.f;
        });
    }
#pragma unroll
    for (int t = 0; t < HR; ++t) x[t] += d[t];
}

// Truncated Pade line derivative of the streamed line window f for this
// lane's HR outputs (output t uses f[t + 1 .. t + PADE_TAPS]).  Interior
// windows run tap-outer so that one tap is live at a time; each output still
// accumulates its taps in ascending order.  Windows near the line ends take
// their rows from the boundary table.
template <int HR, int NPOS>
__device__ __forceinline__ void line_fir(bool fast, const PadeLine& L, int mfirst, CDouble* tc,
                                         const double (&f)[NPOS], double (&out)[HR])
{
    if (fast) {
#pragma unroll
        for (int t = 0; t < HR; ++t) out[t] = 0.0;
#pragma unroll
        for (int u = 0; u < PADE_TAPS; ++u) {
            const double c = tc[u];
#pragma unroll
            for (int t = 0; t < HR; ++t) out[t] = fma(c, f[t + 1 + u], out[t]);
        }
    } else {
#pragma unroll
        for (int t = 0; t < HR; ++t) {
            const int m = mfirst + t;
            double a = 0.0;
            if (m >= 0 && m < L.n_out) {
                CDouble* cr = as_const(pade_row(L, m));
#pragma unroll
                for (int u = 0; u < PADE_TAPS; ++u) a = fma(cr[u], f[t + 1 + u], a);
            }
            out[t] = a;
        }
    }
}

template <int K, int MODE, class S, int FORM = FORM_FP64>
__device__ __forceinline__ void col_tile(const ColArgs& a, const Coef& cf, const PadeTaps& taps,
                                         const PadeLine& L, const ChebSchedule& cs, int bxi, int byi)
{
    constexpr int CW = S::CW, CWP = S::CWP, NL = S::NL, NTC = S::NTC;
    constexpr int TR = ColShape<K, S>::TR;          // region rows
    constexpr int OH = ColShape<K, S>::OH;          // output rows
    constexpr int HR = ColShape<K, S>::HR;          // rows per lane
    constexpr int HALO_X = K + 1;                   // column halo (one more for the cross-line term)
    constexpr bool YPART = MODE != COL_HY;
    constexpr bool SPLIT = MODE == COL_E_TRACKED || MODE == COL_E_DISCRETE || MODE == COL_HX_DISCRETE;
    constexpr bool ESTEP = MODE == COL_E_TRACKED || MODE == COL_E_DISCRETE;
    constexpr int NPOS = HR + PADE_TAPS - 1 + 2;    // streamed line positions (+1 each side for G)
    // LDS: the column sums [TR][CWP], the rows next to the part splits
    // [parity][part][first/last][column], and with the carried Laplacian the
    // curl of H on the output rows [TR][CW] (kept out of registers during
    // the solve).
    constexpr bool PARK_CV = MODE == COL_E_TRACKED && FORM != FORM_RHS;
    constexpr int LDS_DOUBLES = TR * CWP + (FORM == FORM_RHS ? 0 : 2 * NL * 2 * CW) + (PARK_CV ? TR * CW : 0);
    __shared__ double lds_all[LDS_DOUBLES];
    double* lds = lds_all;
    double* bnd = lds_all + TR * CWP;
    double* cvb = bnd + (FORM == FORM_RHS ? 0 : 2 * NL * 2 * CW);

    const int tid = threadIdx.x;
    const int lane = tid % CW;                      // region column
    const int part = tid / CW;                      // rows [part HR, (part+1) HR)
    const int rbase = part * HR;
    const int ow = CW - 2 * HALO_X;
    const UGrid& g = a.g;
    const int x0 = g.lo[0] + bxi * ow;
    const int y0 = g.lo[1] + byi * OH;
    const int gx = x0 - HALO_X + lane;
    const int P = a.P, N = a.N;
    const bool col_active = gx >= g.lo[0] && gx < g.hi[0];
    for (int e = tid; e < TR; e += NTC) {
        lds[e * CWP] = 0.0;
        lds[e * CWP + CW + 1] = 0.0;
    }
    double* my = lds + lane + 1 + rbase * CWP;      // this lane's first row

    double r[HR];            // right-hand side, then the Chebyshev residual
    double cv[HR];           // carried Laplacian: curl^A H on this lane's rows

    // ---------------- right-hand side ----------------
    if (YPART) {
        const int n_in = L.n_in;
        const int mofs = ESTEP ? 1 : 0;                     // gy = m + mofs
        const int mfirst = y0 - K + rbase - mofs;           // Pade output index of this lane's row 0
        const int gfirst = mfirst - PADE_R - 1;             // first streamed position
        const bool col_data = gx >= 0 && gx <= N;           // a stored column (walls included)
        const bool half_line = ESTEP;
        const bool fast = pade_interior(L, mfirst < 0 ? 0 : mfirst, mfirst + HR - 1);
        const double* colp = a.src + gx;
        // interior taps: the table row after the boundary rows, read through
        // the constant address space so the uniform loads go to SGPRs
        const CDouble* tc = as_const(L.rows + (L.all ? 0 : (size_t)(2 * L.b) * PADE_TAPS));
        double f[NPOS];
#pragma unroll
        for (int p = 0; p < NPOS; ++p) {
            const int gg = gfirst + p;
            f[p] = (col_data && gg >= 0 && gg < n_in) ? colp[gg * P] : 0.0;
        }
        if (SPLIT) {
            // raw line derivative P: its second difference across lines
            // completes G; with the carried Laplacian it is also curl^A H
            line_fir<HR>(fast, L, mfirst, tc, f, cv);
#pragma unroll
            for (int t = 0; t < HR; ++t) my[t * CWP] = cv[t];
            // in place: f -> alpha f + (second difference along the line) / 12;
            // half-point lines take even ghosts at their ends, node lines of
            // E vanish on the walls
            double prevf = 0.0;
#pragma unroll
            for (int p = 0; p < NPOS; ++p) {
                const int gg = gfirst + p;
                const double cur = f[p];
                double lo = prevf, hi = (p < NPOS - 1) ? f[p + 1] : 0.0;
                if (half_line) {
                    if (gg == 0) lo = cur;
                    if (gg == n_in - 1) hi = cur;
                }
                double v = fma(cf.alpha, cur, (lo + hi - 2.0 * cur) * (1.0 / 12.0));
                if (gg < 0 || gg >= n_in || !col_data) v = 0.0;
                if (!half_line && (gg == 0 || gg == n_in - 1)) v = 0.0;
                f[p] = v;
                prevf = cur;
            }
        }
        // line derivative of the conditioned input
        line_fir<HR>(fast, L, mfirst, tc, f, r);
        if (SPLIT) {
            __syncthreads();
            // cross-line part of G: (P(x-1) + P(x+1) - 2 P(x)) / 12
#pragma unroll
            for (int t = 0; t < HR; ++t) {
                const double* q = my + t * CWP;
                r[t] += (q[-1] + q[1] - 2.0 * q[0]) * (1.0 / 12.0);
            }
            __syncthreads();
        }
    }

    // combine with the precomputed part and mask to the unknowns
    const double ysign = ESTEP ? -cf.z : (MODE == COL_HY ? 0.0 : -1.0 / cf.z);
#pragma unroll
    for (int t = 0; t < HR; ++t) {
        const int gy = y0 - K + rbase + t;
        const bool act = col_active && gy >= g.lo[1] && gy < g.hi[1];
        double v = 0.0;
        if (act) {
            const size_t o = (size_t)gy * P + gx;
            v = YPART ? ysign * r[t] : 0.0;
            if (a.t0) v += a.t0[o];
        }
        r[t] = v;
    }
    if (MODE == COL_E_TRACKED) {
#pragma unroll
        for (int t = 0; t < HR; ++t) {
            const int row = rbase + t;
            const int gy = y0 - K + row;
            double v = 0.0;
            if (row >= K && row < K + OH && col_active && gy < g.hi[1]) v = a.t1[(size_t)gy * P + gx] - cv[t];
            cv[t] = v;
            if (PARK_CV) cvb[row * CW + lane] = v;
        }
    }

    if (FORM == FORM_RHS) {
        if (lane < HALO_X || lane >= CW - HALO_X || !col_active) return;
#pragma unroll
        for (int t = 0; t < HR; ++t) {
            const int row = rbase + t;
            if (row < K || row >= K + OH) continue;
            const int gy = y0 - K + row;
            if (gy >= g.hi[1]) continue;
            const size_t o = (size_t)gy * P + gx;
            a.b_out[o] = r[t];
            if (MODE == COL_E_TRACKED) a.cv_out[o] = cv[t];
        }
        return;
    }

    // ---------------- solve M Phi = b (b in r[]) ----------------
    const bool nx = g.neumann[0], ny = g.neumann[1];
    const int rx0 = x0 - HALO_X, ry0 = y0 - K;
    ColCtx ctx;
    ctx.inner = rx0 > g.lo[0] && rx0 + CW < g.hi[0] && ry0 > g.lo[1] && ry0 + TR < g.hi[1];
    ctx.mirror_lo_x = nx && gx == g.lo[0];
    ctx.mirror_hi_x = nx && gx == g.hi[0] - 1;
    ctx.col_active = col_active;
    ctx.ny = ny;
    ctx.gy0 = ry0 + rbase;
    ctx.ylo = g.lo[1];
    ctx.yhi = g.hi[1];
    ctx.part = part;
    ctx.lane = lane;
    double phi[HR];
    if (FORM == FORM_FP64) {
        // Chebyshev on [alpha, alpha + 16/3 beta] in FP64, K applications;
        // L9 d = (S(x-1) + S(x+1) + 4 S(x) - 36 d) / 6, A d = alpha d - beta L9 d
        const double b6 = cf.beta * (1.0 / 6.0);
        const double a36 = fma(36.0, b6, cf.alpha);
        const bool at_lo_x = gx == g.lo[0], at_hi_x = gx == g.hi[0] - 1;
        const bool inner = ctx.inner;
        double d[HR], xs[HR], sown[HR];
#pragma unroll
        for (int t = 0; t < HR; ++t) {
            d[t] = r[t] * cs.inv_theta;
            xs[t] = 0.0;
        }
        bnd[(part * 2 + 0) * CW + lane] = d[0];
        bnd[(part * 2 + 1) * CW + lane] = d[HR - 1];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double* bp = bnd + (k & 1) * (NL * 2 * CW);
            double* bq = bnd + ((k & 1) ^ 1) * (NL * 2 * CW);
            const double above = part > 0 ? bp[((part - 1) * 2 + 1) * CW + lane] : 0.0;
            const double below = part < NL - 1 ? bp[((part + 1) * 2 + 0) * CW + lane] : 0.0;
            const double c1 = cs.c1[k], c2 = cs.c2[k];
            if (inner) {
#pragma unroll
                for (int t = 0; t < HR; ++t) {
                    const double up = t > 0 ? d[t - 1] : above;
                    const double dn = t < HR - 1 ? d[t + 1] : below;
                    sown[t] = fma(4.0, d[t], up + dn);
                    my[t * CWP] = sown[t];
                }
                __syncthreads();
#pragma unroll
                for (int t = 0; t < HR; ++t) {
                    const double* q = my + t * CWP;
                    const double dc = d[t];
                    const double ad = fma(a36, dc, -b6 * fma(4.0, sown[t], q[-1] + q[1]));
                    xs[t] += dc;
                    r[t] -= ad;
                    d[t] = fma(c1, dc, c2 * r[t]);
                }
            } else {
#pragma unroll
                for (int t = 0; t < HR; ++t) {
                    const int gy = ry0 + rbase + t;
                    double up = t > 0 ? d[t - 1] : above;
                    double dn = t < HR - 1 ? d[t + 1] : below;
                    if (ny && gy == g.lo[1]) up = d[t];
                    if (ny && gy == g.hi[1] - 1) dn = d[t];
                    sown[t] = fma(4.0, d[t], up + dn);
                    my[t * CWP] = sown[t];
                }
                __syncthreads();
#pragma unroll
                for (int t = 0; t < HR; ++t) {
                    const int gy = ry0 + rbase + t;
                    const double* q = my + t * CWP;
                    const double sc = sown[t];
                    double sl = q[-1], sr = q[1];
                    if (nx && at_lo_x) sl = sc;
                    if (nx && at_hi_x) sr = sc;
                    const double dc = d[t];
                    const double ad = fma(a36, dc, -b6 * fma(4.0, sc, sl + sr));
                    const bool act = col_active && gy >= g.lo[1] && gy < g.hi[1];
                    xs[t] += dc;
                    const double rn = r[t] - ad;
                    r[t] = act ? rn : 0.0;
                    d[t] = act ? fma(c1, dc, c2 * rn) : 0.0;
                }
            }
            bq[(part * 2 + 0) * CW + lane] = d[0];
            bq[(part * 2 + 1) * CW + lane] = d[HR - 1];
            __syncthreads();
        }
#pragma unroll
        for (int t = 0; t < HR; ++t) phi[t] = xs[t] + d[t];
    } else {
        // two FP32 Chebyshev rounds with an FP64 residual between them:
        // x1 = C(b), res = b - M x1 (FP64), Phi = x1 + C(res)
        constexpr int K1 = (K - 1) / 2, K2 = K - 1 - K1;
        float* ldsf = reinterpret_cast<float*>(lds);
        float* bndf = reinterpret_cast<float*>(bnd);
        float x1[HR];
        cheb32<HR, S, K1>(ctx, r, x1, ldsf, bndf, cf, cs);
        double xd[HR];
#pragma unroll
        for (int t = 0; t < HR; ++t) xd[t] = (double)x1[t];
        apply_m<HR, S>(ctx, xd, lds, bnd, cf.alpha, cf.beta,
                       [&](int t, double m, bool act) { r[t] = act ? r[t] - m : 0.0; });
        float x2[HR];
        cheb32<HR, S, K2>(ctx, r, x2, ldsf, bndf, cf, cs);
#pragma unroll
        for (int t = 0; t < HR; ++t) phi[t] = (double)x1[t] + (double)x2[t];
    }

    // ---------------- update ----------------
    if (lane < HALO_X || lane >= CW - HALO_X || !col_active) return;
#pragma unroll
    for (int t = 0; t < HR; ++t) {
        const int row = rbase + t;
        if (row < K || row >= K + OH) continue;
        const int gy = y0 - K + row;
        if (gy >= g.hi[1]) continue;
        const size_t o = (size_t)gy * P + gx;
        const double de = cf.cfl * phi[t];
        a.field[o] += de;
        if (MODE == COL_E_TRACKED) a.ge[o] += fma(cf.ge_gain, de, -cf.ge_curl * cvb[row * CW + lane]);
    }
}

// XCD-aware tile order.  Workgroup IDs of a launch are dealt to the XCDs in
// turn (ID mod 8), and each XCD has its own L2.  XCD x takes the x-th
// contiguous range of the tile sequence, so tiles that share halo data run
// at about the same time on the same L2.  The grid has 8 ceil(T/8) groups;
// the few past the last tile return at once.
constexpr int NXCD = 8;
__host__ __device__ inline int xcd_grid(int tiles) { return NXCD * ((tiles + NXCD - 1) / NXCD); }
__device__ __forceinline__ bool xcd_tile(int tiles, int& l)
{
    const int per = (tiles + NXCD - 1) / NXCD;
    const int id = (int)blockIdx.x;
    l = (id % NXCD) * per + id / NXCD;
    return l < tiles;
}

// Tile counts of the two 2D kernels.
__host__ __device__ inline int xlines_tiles_x(int n_out) { return (n_out + XT_OUT - 1) / XT_OUT; }
__host__ __device__ inline int xlines_tiles_y(int N) { return (N - 1 + XT_ROWS - 1) / XT_ROWS; }
template <int K, class S>
__host__ __device__ inline int col_tiles_x(const UGrid& g)
{
    return (g.hi[0] - g.lo[0] + S::CW - 2 * (K + 1) - 1) / (S::CW - 2 * (K + 1));
}
template <int K, class S>
__host__ __device__ inline int col_tiles_y(const UGrid& g)
{
    return (g.hi[1] - g.lo[1] + ColShape<K, S>::OH - 1) / ColShape<K, S>::OH;
}

// Dispatch a callable templated on (K, shape) from run-time values; shapes
// 1 and 2 exist for K in 4..6 only (shape 0 otherwise).
template <class F>
inline auto with_k_shape(int K, int shape, F&& f)
{
    if (shape == 1 && K >= 4 && K <= 6) {
        if (K == 4) return f.template operator()<4, Shape1>();
        if (K == 5) return f.template operator()<5, Shape1>();
        return f.template operator()<6, Shape1>();
    }
    if (shape == 2 && K >= 4 && K <= 6) {
        if (K == 4) return f.template operator()<4, Shape2>();
        if (K == 5) return f.template operator()<5, Shape2>();
        return f.template operator()<6, Shape2>();
    }
    switch (K) {
        case 1: return f.template operator()<1, Shape0>();
        case 2: return f.template operator()<2, Shape0>();
        case 3: return f.template operator()<3, Shape0>();
        case 4: return f.template operator()<4, Shape0>();
        case 5: return f.template operator()<5, Shape0>();
        case 6: return f.template operator()<6, Shape0>();
        case 7: return f.template operator()<7, Shape0>();
        default: return f.template operator()<8, Shape0>();
    }
}

// Mixed precision: the tile halo K = 2 s + 1 for s FP32 sweeps per round;
// instantiated for s = 1, 2, 3 with the default shape.
template <class F>
inline auto with_k_mixed(int K, F&& f)
{
    if (K <= 3) return f.template operator()<3, Shape0>();
    if (K <= 5) return f.template operator()<5, Shape0>();
    return f.template operator()<7, Shape0>();
}

// unknowns of the 2D components
__host__ __device__ inline UGrid ugrid_ez(int N) { return UGrid{{1, 1, 0}, {N, N, 1}, {0, 0, 0}}; }
__host__ __device__ inline UGrid ugrid_hx(int N) { return UGrid{{1, 0, 0}, {N, N, 1}, {0, 1, 0}}; }
__host__ __device__ inline UGrid ugrid_hy(int N) { return UGrid{{0, 1, 0}, {N, N, 1}, {1, 0, 0}}; }

}  // namespace c4m
