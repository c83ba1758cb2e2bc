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
//     neighbouring columns) and the x-line part: in Step 1 formed here from
//     the raw x-line derivative P of the row and its neighbours (the
//     conditioning commutes with the interior rows of the x-lines too; the
//     columns near the x ends read it from the x-line pass), in Step 2
//     precomputed;
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
// (bound_ctrl: a lane without a source lane reads zero)
__device__ __forceinline__ double from_left(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_right(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x130, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

constexpr int SW_COLS = 64;          // columns of a strip (one wavefront)
constexpr int SW_WIN = COND_TAPS;    // raw rows in the Pade window
constexpr int SW_WAVES = 4;          // strips per workgroup

// Strip shapes: unrolled U steps at a time, per-row inputs fetched LA steps
// ahead.  The region rows TR (a multiple of U; OH = TR - 2 K output rows)
// are chosen per launch so that the strips fill the machine in whole rounds.
template <int K, int MODE, int U, int LA>
struct StripShape {
    static constexpr bool YPART = MODE != COL_HY;
    static constexpr bool SPLIT = MODE == COL_E_TRACKED || MODE == COL_E_DISCRETE || MODE == COL_HX_DISCRETE;
    static constexpr bool ESTEP = MODE == COL_E_TRACKED || MODE == COL_E_DISCRETE;
    // Step 1: the x-line part T0 is formed from the raw x-derivative P (t1)
    // of the row and its neighbours, and read from t0 on the band columns
    static constexpr bool PSRC = ESTEP;
    static constexpr bool HAS_T0 = MODE == COL_HY;
    static constexpr bool CARRY = MODE == COL_E_TRACKED;
    static constexpr int HX = K + (SPLIT ? 1 : 0);   // halo columns on each side
    static constexpr int OW = SW_COLS - 2 * HX;     // output columns
    static constexpr int NW = YPART ? SW_WIN + LA : 1;
    static constexpr int NQ = LA + 1;               // per-row prefetch queue
    static_assert(OW > 0, "strip too narrow for K");
    static_assert(!CARRY || PSRC, "the carried update takes P from the Step 1 stream");
    static_assert(U % 4 == 0, "the boundary form runs 4 steps per block");
};

// Band of Pade rows near each end of the y-lines whose derivatives a
// strip takes from a table pass (k_yband) instead of its interior pair
// form: rows m <= b and m >= n_out - 1 - b (every row of a short line).
// Layout: yb[((q * 2 + e) * YB_ROWS + r) * P + gx], q = 0 raw, 1
// conditioned; e = 0 low end (m = r), 1 high end (m = n_out - rows + r).
__host__ __device__ inline int band_rows(const PadeLine& L) { return L.all ? L.n_out : L.b + 1; }

template <class SS>
__host__ __device__ inline int strip_tiles_x(const UGrid& g)
{
    return (g.hi[0] - g.lo[0] + SS::OW - 1) / SS::OW;
}
__host__ __device__ inline int strip_tiles_y(const UGrid& g, int oh)
{
    return (g.hi[1] - g.lo[1] + oh - 1) / oh;
}

// Buffer (MUBUF) accesses with the hardware range check: a lane whose
// offset is BUF_NULL (beyond every array's byte size, which stays below
// 2^32 - 16 for the 2D sizes accepted) reads 0 and its store is dropped,
// so masked accesses need no branch and an unrolled block of steps stays
// one basic block.
constexpr unsigned BUF_NULL = 0xFFFFFFF0u;
typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const double* p, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
// per-lane offset voff plus a wave-uniform offset soff (only where every
// lane's access is in range)
__device__ __forceinline__ double buf_ld_s(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, off, 0, 0);
}

// The arrays a strip reads and writes (null pointers skipped), as one
// byte range: every 2D array has N + 1 rows of P doubles.
struct StripSpan {
    const double* base;
    unsigned bytes;
    __host__ __device__ unsigned delta(const double* p) const
    {
        return p ? (unsigned)((const char*)p - (const char*)base) : 0u;
    }
};
__host__ __device__ inline size_t strip_span_bytes(const ColArgs& a, const double*& base)
{
    const double* ptrs[6] = {a.src, a.t0, a.t1, a.field, a.ge, a.yb};
    const size_t arr = (size_t)(a.N + 1) * (size_t)a.P * sizeof(double);
    const size_t band = (size_t)4 * YB_ROWS * (size_t)a.P * sizeof(double);
    uintptr_t lo = ~(uintptr_t)0, hi = 0;
    for (int i = 0; i < 6; ++i) {
        if (!ptrs[i]) continue;
        const uintptr_t p = (uintptr_t)ptrs[i];
        lo = p < lo ? p : lo;
        const uintptr_t end = p + (i == 5 ? band : arr);
        hi = end > hi ? end : hi;
    }
    base = (const double*)lo;
    return (size_t)(hi - lo);
}
__host__ __device__ inline StripSpan strip_span(const ColArgs& a)
{
    StripSpan s;
    s.bytes = (unsigned)strip_span_bytes(a, s.base);
    return s;
}

// One strip: region columns gx = x0 - HX + lane, output rows [y0, y0 + TR - 2K).
// XB: some lanes of the strip lie on or beyond the x ends of the unknowns
// (lane masks, Neumann mirrors, zero source off the stored columns).
// YB: some region rows lie on or beyond the y ends, or some Pade rows of the
// region are in the end bands (row masks and mirrors; band derivatives from
// the table pass).  Elsewhere the interior (Toeplitz) Pade rows apply, in
// pair form.  UU steps per unrolled block.
// Every load goes to an address inside its array (rows and columns clamped,
// values outside replaced afterwards), stores of masked lanes are dropped by
// the buffer range check.
template <int K, int MODE, int U, int LA, bool XB, bool YB, int UU>
__device__ __forceinline__ void strip_run(const ColArgs& a, const Coef& cf, const PadeLine& L,
                                          const ChebSchedule& cs, int x0, int y0, const int TR, const bool rev)
{
    using SS = StripShape<K, MODE, U, LA>;
    constexpr bool YPART = SS::YPART, SPLIT = SS::SPLIT, HAS_T0 = SS::HAS_T0, CARRY = SS::CARRY;
    constexpr bool PSRC = SS::PSRC;
    constexpr int HX = SS::HX, NQ = SS::NQ;
    // the raw derivative of row m + 1 needs rows m - 11 .. m + 14 only
    constexpr int W0 = YPART ? 2 : 0;
    constexpr int NW = SS::NW - W0;
    const int lane = (int)(threadIdx.x % SW_COLS);
    const UGrid& g = a.g;
    const int P = a.P, N = a.N;
    const int gx = x0 - HX + lane;
    const bool col_active = !XB || (gx >= g.lo[0] && gx < g.hi[0]);
    const bool col_data = !XB || (gx >= 0 && gx <= N);
    const bool nx = g.neumann[0], ny = g.neumann[1];
    const bool mlo = XB && nx && gx == g.lo[0], mhi = XB && nx && gx == g.hi[0] - 1;
    const bool lane_out = lane >= HX && lane < SW_COLS - HX && col_active;
    const int ylo = g.lo[1], yhi = g.hi[1];
    const int ry0 = y0 - K;                             // grid row of the region's first row
    const int mofs = SS::ESTEP ? 1 : 0;                 // grid row = Pade output index + mofs
    // Walking direction: down (rev false) or up.  Step ry takes region row
    // ry from the walking start; rows behind in walking order are above
    // (down) or below (up).  Segments of a strip alternate, so the rows
    // two neighbouring segments share are read by both at about the same
    // time (both at their starts or both at their ends).
    const int dir = rev ? -1 : 1;
    const int gy0 = rev ? ry0 + TR - 1 : ry0;          // grid row of step 0
    const int mfirst = gy0 - mofs;                      // its Pade output index
    // window slot i after the load of step ry holds raw row wbase + dir (ry + i);
    // the pair form over slots 0..25 is dir P(m + dir), m = mfirst + dir ry
    const int wbase = rev ? mfirst + (SW_WIN / 2 - 2) : mfirst - (SW_WIN / 2 - 3);
    const double psg = rev ? -1.0 : 1.0;
    const int n_in = L.n_in, n_out = L.n_out;
    // Step 1: columns whose x-line output (m = gx - 1; the grid is square, so
    // the x-lines share the y-lines' line) lies in an end band take T0 from
    // the x-line pass
    const int mx = gx - 1;
    const bool xband = PSRC && XB && col_active && (L.all || mx <= L.b || mx >= n_out - 1 - L.b);

    // one buffer over every array of the strip (their span stays below
    // BUF_NULL: the caller takes the strip form only then); each array is a
    // byte offset in it
    const StripSpan sp = strip_span(a);
    const __amdgpu_buffer_rsrc_t rb = buf_rsrc(sp.base, sp.bytes);
    const unsigned dsrc = sp.delta(a.src), dt0 = sp.delta(a.t0), dt1 = sp.delta(a.t1);
    const unsigned dfield = sp.delta(a.field), dge = sp.delta(a.ge);
    const unsigned rowb = (unsigned)P * (unsigned)sizeof(double);
    const int gxc = gx < 0 ? 0 : (gx > N ? N : gx);
    const unsigned laneb = (unsigned)gxc * (unsigned)sizeof(double);
    auto clampi = [](int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); };

    const double b6 = cf.beta * (1.0 / 6.0);
    const double a36 = fma(36.0, b6, cf.alpha);
    const double ysign = SS::ESTEP ? -cf.z : (MODE == COL_HY ? 0.0 : -1.0 / cf.z);

    // raw source row gg (zero off the stored columns; rows off the line only
    // feed derivatives of band rows, which are replaced)
    auto load_raw = [&](int gg) -> double {
        const double v = buf_ld_s(rb, laneb, dsrc + (unsigned)(YB ? clampi(gg, 0, n_in - 1) : gg) * rowb);
        return col_data ? v : 0.0;
    };
    // band values (q = 0 raw, 1 conditioned) of Pade row m, zero off the line
    const int nbr = band_rows(L);
    const unsigned dyb = sp.delta(a.yb);
    auto in_band = [&](int m) -> bool { return YB && (m <= L.b || m >= n_out - 1 - L.b || L.all); };
    auto band = [&](int q, int m) -> double {
        const int e = m < nbr ? 0 : 1;
        const int r = clampi(e ? m - (n_out - nbr) : m, 0, nbr - 1);
        const double v = buf_ld_s(rb, laneb, dyb + (unsigned)((q * 2 + e) * YB_ROWS + r) * rowb);
        return (m >= 0 && m < n_out && col_data) ? v : 0.0;
    };
    auto row_in = [&](int gy) -> bool { return !YB || (gy >= ylo && gy < yhi); };
    auto grow = [&](int ry) -> int { return gy0 + dir * ry; };   // grid row of step ry
    auto out_row = [&](int ry) -> bool {   // step ry updates grid row grow(ry) - dir K
        return ry >= 2 * K && ry < TR && (!YB || grow(ry) - dir * K < yhi);
    };
    // Step 1: raw x-line derivative P of the row of step r (rows clamped
    // into 0..N, where the x-line pass stores it)
    auto load_p = [&](int r) -> double {
        const int gg = YB ? clampi(grow(r), ylo - 1, yhi) : grow(r);
        const double v = buf_ld_s(rb, laneb, dt1 + (unsigned)gg * rowb);
        return col_data ? v : 0.0;
    };
    // per-row inputs: t0 of the row of step ry (Step 1: P of the row of step
    // ry + 1, and in t1v T0 of the band columns of the row of step ry);
    // field and G_E of the output row that leaves the pipeline at step ry
    // (rows clamped into the valid range: values of other rows are never
    // used)
    auto prefetch = [&](int ry, double& t0v, double& fv, double& gv, double& t1v) {
        const int rt = ry < TR ? ry : TR - 1;
        const int gyt = YB ? clampi(grow(rt), ylo, yhi - 1) : grow(rt);
        t0v = HAS_T0 ? buf_ld_s(rb, laneb, dt0 + (unsigned)gyt * rowb) : 0.0;
        if (PSRC) t0v = load_p(ry + 1 < TR ? ry + 1 : TR);
        const int ro = rt < 2 * K ? 2 * K : rt;
        const int gyo = YB ? clampi(grow(ro) - dir * K, ylo, yhi - 1) : grow(ro) - dir * K;
        const unsigned so = (unsigned)gyo * rowb;
        fv = buf_ld_s(rb, laneb, dfield + so);
        gv = CARRY ? buf_ld_s(rb, laneb, dge + so) : 0.0;
        t1v = (PSRC && XB) ? buf_ld(rb, xband ? dt0 + (unsigned)gyt * rowb + laneb : BUF_NULL) : 0.0;
    };

    // ---- state
    double fw[NW];                 // raw window (see wbase)
    double t0q[NQ], fq[NQ], gq[NQ], t1q[NQ];
    // carried Laplacian: raw curl of the last K + 1 rows (x-line minus y-line
    // raw derivative)
    double pd[K + 1];
    double dp1[K], dp2[K], rp1[K], xp1[K];
#pragma unroll
    for (int j = 0; j < K; ++j) dp1[j] = dp2[j] = rp1[j] = xp1[j] = 0.0;
#pragma unroll
    for (int j = 0; j <= K; ++j) pd[j] = 0.0;
    // Step 1: P of the rows of the previous and the current step
    double pprev = PSRC ? load_p(-1) : 0.0, pcur = PSRC ? load_p(0) : 0.0;
    if (YPART) {
#pragma unroll
        for (int i = W0 ? 0 : 1; i < NW; ++i) fw[i] = load_raw(wbase + dir * (i - 1));
    }
#pragma unroll
    for (int i = 1; i < NQ; ++i) prefetch(i - 1, t0q[i], fq[i], gq[i], t1q[i]);

    CDouble* pq = as_const(L.pairs) + COND_TAPS / 2;    // raw interior pair taps
    // interior raw derivative from 26 consecutive rows w(0..25) (rows
    // m - 12 .. m + 13): sum_j p_j (f(m - j) - f(m + 1 + j))
    auto fir_pair = [&](auto&& w) -> double {
        double p0 = 0.0, p1 = 0.0;
#pragma unroll
        for (int j = 0; j < PADE_TAPS / 2; j += 2) {
            p0 = fma(pq[j], w(PADE_TAPS / 2 - 1 - j) - w(PADE_TAPS / 2 + j), p0);
            if (j + 1 < PADE_TAPS / 2) p1 = fma(pq[j + 1], w(PADE_TAPS / 2 - 2 - j) - w(PADE_TAPS / 2 + 1 + j), p1);
        }
        return p0 + p1;
    };
    // raw derivatives of the rows mfirst - dir and mfirst before step 0
    // (fw[i] holds row wbase + dir (i - 1))
    double pm1 = 0.0, pm0 = 0.0;
    if (YPART) {
        const double extra = load_raw(wbase - 2 * dir);
        pm1 = psg * fir_pair([&](int i) { return i == 0 ? extra : fw[i - 1]; });
        pm0 = psg * fir_pair([&](int i) { return fw[i]; });
        if (YB) {
            pm1 = in_band(mfirst - dir) ? band(0, mfirst - dir) : pm1;
            pm0 = in_band(mfirst) ? band(0, mfirst) : pm0;
        }
    }

    for (int blk = 0; blk < TR; blk += UU) {
#pragma unroll
        for (int u = 0; u < UU; ++u) {
            const int ry = blk + u;
            // ---- advance the window and the prefetch queues
            if (YPART) {
#pragma unroll
                for (int i = 0; i < NW - 1; ++i) fw[i] = fw[i + 1];
                fw[NW - 1] = load_raw(wbase + dir * (ry + NW - 1));
            }
#pragma unroll
            for (int i = 0; i < NQ - 1; ++i) {
                t0q[i] = t0q[i + 1];
                fq[i] = fq[i + 1];
                gq[i] = gq[i + 1];
                t1q[i] = t1q[i + 1];
            }
            prefetch(ry + LA, t0q[NQ - 1], fq[NQ - 1], gq[NQ - 1], t1q[NQ - 1]);

            // ---- line derivatives of Pade row m = mfirst + dir ry: raw (pr) and
            // of the conditioned source (cr).  The conditioning along the line
            // commutes with the interior (Toeplitz) rows, so there
            // R(m) = alpha P(m) + (P(m-1) + P(m+1) - 2 P(m)) / 12.
            double pr = 0.0, cr = 0.0;
            if (YPART) {
                const int m = mfirst + dir * ry;
                double pp1 = psg * fir_pair([&](int i2) { return fw[i2]; });
                if (YB) pp1 = in_band(m + dir) ? band(0, m + dir) : pp1;
                pr = pm0;
                if (SPLIT) {
                    cr = fma(cf.alpha, pm0, (pm1 + pp1 - 2.0 * pm0) * (1.0 / 12.0));
                    if (YB) cr = in_band(m) ? band(1, m) : cr;
                } else {
                    cr = pm0;
                }
                pm1 = pm0;
                pm0 = pp1;
            }

            // ---- right-hand side of the row of step ry
            const int gy = grow(ry);
            double b;
            {
                double v = 0.0;
                if (YPART) {
                    double sum = cr;
                    if (SPLIT) sum += (from_left(pr) + from_right(pr) - 2.0 * pr) * (1.0 / 12.0);
                    v = ysign * sum;
                }
                if (HAS_T0) v += t0q[0];
                if (PSRC) {
                    // T0 = Z (alpha P + (P(m-1) + P(m+1) - 2 P) / 12 + (P_s + P_n - 2 P) / 12)
                    const double pn = t0q[0];
                    const double pc = pcur;
                    const double along = fma(cf.alpha, pc, (from_left(pc) + from_right(pc) - 2.0 * pc) * (1.0 / 12.0));
                    const double across = (pprev + pn - 2.0 * pc) * (1.0 / 12.0);
                    double tv = cf.z * (along + across);
                    if (XB) tv = xband ? t1q[0] : tv;
                    v += tv;
                }
                b = (row_in(gy) && col_active) ? v : 0.0;
            }
            if (CARRY) {
#pragma unroll
                for (int j = 0; j < K; ++j) pd[j] = pd[j + 1];
                pd[K] = pcur - pr;
            }
            if (PSRC) {
                pprev = pcur;
                pcur = t0q[0];
            }

            // ---- Chebyshev pipeline: application j + 1 on the row j + 1 steps behind
            double dn[K + 1], rn[K + 1], xn[K + 1];
            dn[0] = b * cs.inv_theta;
            rn[0] = b;
            xn[0] = 0.0;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int gq_ = gy - dir * (j + 1);
                // older row (dp2) and newer row (dn): above and below when
                // walking down, below and above when walking up
                double up = dp2[j], cen = dp1[j], dw = dn[j];
                if (YB) {
                    up = (ny && gq_ == (rev ? yhi - 1 : ylo)) ? cen : up;
                    dw = (ny && gq_ == (rev ? ylo : yhi - 1)) ? cen : dw;
                }
                const double sown = fma(4.0, cen, up + dw);
                double sl = from_left(sown), sr = from_right(sown);
                if (XB) {
                    sl = mlo ? sown : sl;
                    sr = mhi ? sown : sr;
                }
                // r - M d with M d = a36 d - b6 (4 S + S(x-1) + S(x+1))
                xn[j + 1] = j == 0 ? cen : xp1[j] + cen;
                double r_ = fma(b6, fma(4.0, sown, sl + sr), fma(-a36, cen, rp1[j]));
                double d_ = fma(cs.c1[j], cen, cs.c2[j] * r_);
                if (XB || YB) {
                    const bool act = row_in(gq_) && col_active;
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

            // ---- update of grid row gy - dir K (other lanes and rows: BUF_NULL)
            {
                const bool ok = out_row(ry) && lane_out;
                const unsigned row = (unsigned)(gy - dir * K) * rowb + laneb;
                const double de = cf.cfl * (xn[K] + dn[K]);
                buf_st(rb, ok ? dfield + row : BUF_NULL, fq[0] + de);
                if (CARRY)
                    buf_st(rb, ok ? dge + row : BUF_NULL,
                           gq[0] + fma(cf.ge_gain, de, -cf.ge_curl * pd[0]));
            }
        }
    }
}

// Whether every lane of a strip with first region column rx0 lies strictly
// inside the unknowns (no mirror, no mask) and, in Step 1, outside the
// x-line end bands.
template <class SS>
__host__ __device__ inline bool strip_xin(const UGrid& g, const PadeLine& L, int rx0)
{
    bool in = rx0 > g.lo[0] && rx0 + SW_COLS < g.hi[0];
    if (SS::PSRC) in = in && !L.all && rx0 - 1 > L.b && rx0 + SW_COLS - 2 < L.n_out - 1 - L.b;
    return in;
}

// Which form a strip takes: 0 interior, 1 x ends (XB), 2 y ends (XB and YB).
template <class SS, int K>
__host__ __device__ inline int strip_variant(const UGrid& g, const PadeLine& L, int x0, int y0, int tr)
{
    const int rx0 = x0 - SS::HX, ry0 = y0 - K;
    const int mofs = SS::ESTEP ? 1 : 0;
    const bool xin = strip_xin<SS>(g, L, rx0);
    // y: every region row strictly inside; the Pade rows of the region and
    // two beyond each end stay out of the bands, and the window in the line
    bool yin = ry0 > g.lo[1] && ry0 + tr < g.hi[1];
    if (SS::YPART) {
        const int m_lo = ry0 - mofs, m_hi = ry0 - mofs + tr - 1;
        // (either walking direction: the window reaches 14 rows plus the
        // prefetch beyond the region on one side)
        yin = yin && !L.all && m_lo - 2 >= L.b && m_hi + 2 < L.n_out - L.b &&
              m_lo - SW_WIN / 2 - (SS::NW - SW_WIN) >= 0 && m_hi + SW_WIN / 2 + SS::NW - SW_WIN < L.n_in;
    }
    return !yin ? 2 : (!xin ? 1 : 0);
}

// Strip plan: the segments (first output row y0, region rows tr) of the
// strips with some lane at the x ends (type 0: the first xa and the last
// xb strips) and of the other strips (type 1).  Segment lengths are chosen
// so that the estimated work of the items (cost per step of their form
// times steps plus the window fill) is about equal and the items fill whole
// rounds of the resident wave slots.  Items: the type-0 strips first, then
// the type-1 strips, segments of a strip consecutive.
constexpr int STRIP_MAXSEG = 192;
struct StripPlan {
    int strips, xa, xb;
    int nseg[2];
    short y0[2][STRIP_MAXSEG];
    short tr[2][STRIP_MAXSEG];
    __host__ __device__ int items() const
    {
        return (xa + xb) * nseg[0] + (strips - xa - xb) * nseg[1];
    }
    // strip index, output row, region rows and walking direction (odd
    // segments walk up) of item it
    __host__ __device__ void item(int it, int& strip, int& y0v, int& trv, bool& up) const
    {
        const int ix = (xa + xb) * nseg[0];
        int t, k, sg;
        if (it < ix) {
            t = 0;
            k = it / nseg[0];
            sg = it - k * nseg[0];
            strip = k < xa ? k : strips - xb + (k - xa);
        } else {
            t = 1;
            it -= ix;
            k = it / nseg[1];
            sg = it - k * nseg[1];
            strip = xa + k;
        }
        y0v = y0[t][sg];
        trv = tr[t][sg];
        up = (sg & 1) != 0;
    }
};

template <int K, int MODE, int U, int LA>
__device__ __forceinline__ void strip_tile(const ColArgs& a, const Coef& cf, const PadeLine& L,
                                           const ChebSchedule& cs, int x0, int y0, int tr, bool up)
{
    using SS = StripShape<K, MODE, U, LA>;
    const int v = strip_variant<SS, K>(a.g, L, x0, y0, tr);
    if (v == 0)
        strip_run<K, MODE, U, LA, false, false, U>(a, cf, L, cs, x0, y0, tr, up);
    else if (v == 1)
        strip_run<K, MODE, U, LA, true, false, U>(a, cf, L, cs, x0, y0, tr, up);
    else
        strip_run<K, MODE, U, LA, true, true, U>(a, cf, L, cs, x0, y0, tr, up);
}

// Cost model of the plan: work per step of the three forms, the window
// fill in steps, and how many resident waves it takes to keep a SIMD busy
// (the estimated time of a launch is the larger of its longest item and
// its total work over the SIMDs at that many waves each, per round of the
// resident wave slots).
constexpr double STRIP_COST[3] = {1.0, 1.3, 1.9};
constexpr int STRIP_FILL_STEPS = 6;
// (measured at N = 2048: three waves for the strips of both steps; two
// waves were better for Step 1 while its strips read both x-line terms)
template <class SS>
constexpr double strip_waves_per_simd()
{
    return 3.0;
}
template <class SS, int K, int U>
inline bool strip_plan(const UGrid& g, const PadeLine& L, int slots, int simds, StripPlan& plan)
{
    const int strips = strip_tiles_x<SS>(g);
    plan.strips = strips;
    plan.xa = plan.xb = 0;
    auto x0_of = [&](int i) { return g.lo[0] + i * SS::OW; };
    auto xin = [&](int i) { return strip_xin<SS>(g, L, x0_of(i) - SS::HX); };
    while (plan.xa < strips && !xin(plan.xa)) ++plan.xa;
    while (plan.xa + plan.xb < strips && !xin(strips - 1 - plan.xb)) ++plan.xb;
    const int nstr[2] = {plan.xa + plan.xb, strips - plan.xa - plan.xb};
    const int rep[2] = {0, plan.xa};    // a strip of each type
    const int tr_min = ((2 * K + 1) + U - 1) / U * U;
    const int span = g.hi[1] - g.lo[1];
    auto cost = [&](int t, int y0, int tr) {
        return STRIP_COST[strip_variant<SS, K>(g, L, x0_of(rep[t]), y0, tr)] * (tr + STRIP_FILL_STEPS);
    };
    // segments of a strip of type t for a target cost; -1 if too many
    auto layout = [&](int t, double target, bool store, double& worst, double& total) -> int {
        int n = 0;
        for (int y0 = g.lo[1]; y0 < g.hi[1];) {
            int tr = tr_min;
            while (tr + U - 2 * K <= span + 2 * U && cost(t, y0, tr + U) <= target) tr += U;
            const double c = cost(t, y0, tr);
            worst = c > worst ? c : worst;
            total += c * nstr[t];
            if (n == STRIP_MAXSEG) return -1;
            if (store) {
                plan.y0[t][n] = (short)y0;
                plan.tr[t][n] = (short)tr;
            }
            ++n;
            y0 += tr - 2 * K;
        }
        return n;
    };
    double best_t = 0.0, best_make = 0.0;
    for (double t = STRIP_COST[0] * (tr_min + STRIP_FILL_STEPS); t < 1e7; t *= 1.03) {
        double worst = 0.0, total = 0.0;
        int items = 0;
        bool ok = true;
        for (int k = 0; k < 2; ++k) {
            if (!nstr[k]) continue;
            const int n = layout(k, t, false, worst, total);
            if (n < 0) ok = false;
            items += n * nstr[k];
        }
        if (!ok) continue;
        const int rounds = (items + slots - 1) / slots;
        const double per_round = total / rounds / (simds * strip_waves_per_simd<SS>());
        const double make = rounds * (worst > per_round ? worst : per_round);
        if (best_t == 0.0 || make < best_make) {
            best_t = t;
            best_make = make;
        }
        if (items <= slots / 8) break;
    }
    if (best_t == 0.0) return false;
    for (int k = 0; k < 2; ++k) {
        double worst = 0.0, total = 0.0;
        plan.nseg[k] = nstr[k] ? layout(k, best_t, true, worst, total) : 0;
    }
    return true;
}

// Table pass for the strips: raw and conditioned y-line derivatives of
// the band rows of every stored column (one thread per column, band row and
// end), with the exact rows of A^{-1} near the line ends and the end rules
// of the source conditioning folded into the conditioned rows.
template <bool SPLIT>
__device__ __forceinline__ void yband_entry(const double* __restrict__ src, double* __restrict__ yb, int N, int P,
                                            const PadeLine& L, int gx, int r, int e)
{
    const int nbr = band_rows(L), n_out = L.n_out, n_in = L.n_in;
    if (gx > N || r >= nbr || (e == 1 && L.all)) return;
    const int m = e ? n_out - nbr + r : r;
    const int row = pade_row_index(L, m);
    CDouble* tp = as_const(L.rows) + (size_t)row * PADE_TAPS;
    CDouble* tq = as_const(L.crows) + (size_t)row * COND_TAPS;
    double f[COND_TAPS];    // rows m - R - 1 .. m + R + 2, zero off the line
#pragma unroll
    for (int w = 0; w < COND_TAPS; ++w) {
        const int j = m - PADE_R - 1 + w;
        f[w] = (j >= 0 && j < n_in) ? src[(size_t)j * P + gx] : 0.0;
    }
    double pr = 0.0, cr = 0.0;
#pragma unroll
    for (int u = 0; u < PADE_TAPS; ++u) pr = fma(tp[u], f[u + 1], pr);
    if (SPLIT) {
#pragma unroll
        for (int w = 0; w < COND_TAPS; ++w) cr = fma(tq[w], f[w], cr);
    }
    yb[((size_t)(0 * 2 + e) * YB_ROWS + r) * P + gx] = pr;
    yb[((size_t)(1 * 2 + e) * YB_ROWS + r) * P + gx] = SPLIT ? cr : pr;
}

}  // namespace c4m
