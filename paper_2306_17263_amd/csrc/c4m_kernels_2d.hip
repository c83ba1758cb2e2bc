// c4m_kernels_2d.hip -- gfx950 kernels of the 2D TM (Ez, Hx, Hy) step.
//
// One step is four launches:
//   k_rhs_e2d   : b = Z curl^A G(H) at the interior Ez nodes (and, with the
//                 carried Laplacian, c = curl^A H), Step 1 of Section 3.4;
//   k_cheb_2d   : Phi = M^{-1} b by Chebyshev on the closed-form spectral
//                 bounds of M, then Ez += r Phi and G_E += (1+4/r^2) r Phi - (2/r) Z c;
//   k_rhs_h2d   : b_x = -(1/Z) delta_y G_E, b_y = (1/Z) delta_x G_E, Step 2;
//   k_cheb_2d   : Phi = M^{-1} b per H component, H += r Phi.
// G_E = alpha E + l/12 is stored instead of l (the carried Laplacian), so the
// H half-step reads only G_E and H.
//
// Tiles are 64 (x) x 16 (y) outputs per 256-thread workgroup; wave w of a
// workgroup owns rows w, w+4, w+8, w+12 of the tile and lane l column l, so
// every global access of a wave is one contiguous 512-byte row segment.
#include "c4m_internal.h"

namespace c4m {

constexpr int T2X = 64;
constexpr int T2Y = 16;
constexpr int NT2 = 256;
constexpr int RG = NT2 / T2X;            // row groups per workgroup
constexpr int ROWS_PER_THREAD = T2Y / RG;

__device__ __forceinline__ const double* pade_row(const PadeLine& L, int m)
{
    if (L.all) return L.rows + (size_t)m * PADE_TAPS;
    if (m < L.b) return L.rows + (size_t)m * PADE_TAPS;
    if (m >= L.n_out - L.b) return L.rows + (size_t)(m - (L.n_out - L.b) + L.b) * PADE_TAPS;
    return nullptr;
}

// Truncated A^{-1} D applied to an LDS window: s[u * st] holds the line value
// at input index m - PADE_R + u.
__device__ __forceinline__ double fir_taps(const PadeTaps& t, const double* s, int st)
{
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < PADE_TAPS; ++u) acc = fma(t.c[u], s[u * st], acc);
    return acc;
}

__device__ __forceinline__ double fir_row(const double* __restrict__ row, const double* s, int st)
{
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < PADE_TAPS; ++u) acc = fma(row[u], s[u * st], acc);
    return acc;
}

__device__ __forceinline__ double fir_any(const PadeLine& L, const PadeTaps& t, int m, const double* s,
                                          int st)
{
    const double* row = pade_row(L, m);
    return row ? fir_row(row, s, st) : fir_taps(t, s, st);
}

constexpr int XW = T2X + 2 * PADE_R + 2;     // staged width of an x-line window
constexpr int YH = T2Y + 2 * PADE_R + 2;     // staged height of a y-line window
constexpr int STAGE = (T2Y * XW > YH * T2X) ? T2Y * XW : YH * T2X;

// ---------------------------------------------------------------------------
// Step 1 right-hand side.  Output nodes i, j in [1, N-1].
// x part: delta_x of G(Hy) along rows j (Hy at half points 0..N-1 in x,
//         even ghosts at both ends), N-1 outputs at the interior nodes.
// y part: delta_y of G(Hx) along columns i (Hx at half points in y).
// G u = alpha u + (u_W + u_E + u_S + u_N - 4 u)/12 with the same ghosts along
// the half axis and the stored wall values along the node axis.
// ---------------------------------------------------------------------------
template <bool TRACKED>
__global__ __launch_bounds__(NT2) void k_rhs_e2d(const double* __restrict__ hx,
                                                  const double* __restrict__ hy,
                                                  double* __restrict__ b, double* __restrict__ c,
                                                  int N, int P, Coef cf, PadeTaps taps, PadeLine L)
{
    __shared__ double sg[STAGE];
    __shared__ double sh[TRACKED ? STAGE : 1];
    const int tid = threadIdx.x;
    const int col = tid % T2X;
    const int rg = tid / T2X;
    const int i0 = 1 + blockIdx.x * T2X;
    const int j0 = 1 + blockIdx.y * T2Y;
    const int nout = N - 1;
    double accb[ROWS_PER_THREAD], accc[ROWS_PER_THREAD];

    // ---- x part ----
    const int mx0 = i0 - 1;
    for (int e = tid; e < T2Y * XW; e += NT2) {
        const int rr = e / XW, q = e - rr * XW;
        const int j = j0 + rr, g = mx0 - PADE_R + q;
        double vh = 0.0, vg = 0.0;
        if (j <= N - 1 && g >= 0 && g < N) {
            const double* row = hy + (size_t)j * P;
            const double h0 = row[g];
            const double hl = row[g > 0 ? g - 1 : 0];
            const double hr = row[g < N - 1 ? g + 1 : N - 1];
            const double hs = hy[(size_t)(j - 1) * P + g];
            const double hn = hy[(size_t)(j + 1) * P + g];
            vh = h0;
            vg = fma(cf.alpha, h0, (hl + hr + hs + hn - 4.0 * h0) * (1.0 / 12.0));
        }
        sg[e] = vg;
        if (TRACKED) sh[e] = vh;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < ROWS_PER_THREAD; ++t) {
        const int rr = rg + RG * t;
        const int m = mx0 + col;
        double vb = 0.0, vc = 0.0;
        if (m < nout) {
            const double* row = pade_row(L, m);
            if (row) {
                vb = fir_row(row, sg + rr * XW + col, 1);
                if (TRACKED) vc = fir_row(row, sh + rr * XW + col, 1);
            } else {
                vb = fir_taps(taps, sg + rr * XW + col, 1);
                if (TRACKED) vc = fir_taps(taps, sh + rr * XW + col, 1);
            }
        }
        accb[t] = vb;
        accc[t] = vc;
    }
    __syncthreads();

    // ---- y part ----
    const int my0 = j0 - 1;
    for (int e = tid; e < YH * T2X; e += NT2) {
        const int q = e / T2X, cc = e - q * T2X;
        const int i = i0 + cc, g = my0 - PADE_R + q;
        double vh = 0.0, vg = 0.0;
        if (i <= N - 1 && g >= 0 && g < N) {
            const double h0 = hx[(size_t)g * P + i];
            const double hs = hx[(size_t)(g > 0 ? g - 1 : 0) * P + i];
            const double hn = hx[(size_t)(g < N - 1 ? g + 1 : N - 1) * P + i];
            const double hl = hx[(size_t)g * P + i - 1];
            const double hr = hx[(size_t)g * P + i + 1];
            vh = h0;
            vg = fma(cf.alpha, h0, (hl + hr + hs + hn - 4.0 * h0) * (1.0 / 12.0));
        }
        sg[e] = vg;
        if (TRACKED) sh[e] = vh;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < ROWS_PER_THREAD; ++t) {
        const int rr = rg + RG * t;
        const int m = my0 + rr;
        const int j = j0 + rr, i = i0 + col;
        if (m < nout) {
            const double vy = fir_any(L, taps, m, sg + rr * T2X + col, T2X);
            const double vyh = TRACKED ? fir_any(L, taps, m, sh + rr * T2X + col, T2X) : 0.0;
            if (j <= N - 1 && i <= N - 1) {
                b[(size_t)j * P + i] = cf.z * (accb[t] - vy);
                if (TRACKED) c[(size_t)j * P + i] = accc[t] - vyh;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Step 2 right-hand sides from G_E (stored, or alpha E + L5 E / 12 in the
// DISCRETE variant; zero on the walls either way).
// z = 0: b_x(j, i) = -(1/Z) delta_y G_E along column i, i in [1, N-1], j in [0, N-1].
// z = 1: b_y(j, i) = +(1/Z) delta_x G_E along row j,    j in [1, N-1], i in [0, N-1].
// ---------------------------------------------------------------------------
template <bool TRACKED>
__device__ __forceinline__ double ge_value(const double* __restrict__ src, int j, int i, int N, int P,
                                           double alpha)
{
    if (TRACKED) return src[(size_t)j * P + i];
    if (i == 0 || i == N || j == 0 || j == N) return 0.0;
    const double* p = src + (size_t)j * P + i;
    const double e0 = p[0];
    return fma(alpha, e0, (p[-1] + p[1] + p[-P] + p[P] - 4.0 * e0) * (1.0 / 12.0));
}

template <bool TRACKED>
__global__ __launch_bounds__(NT2) void k_rhs_h2d(const double* __restrict__ src,
                                                  double* __restrict__ bx, double* __restrict__ by,
                                                  int N, int P, Coef cf, PadeTaps taps, PadeLine L)
{
    __shared__ double sg[STAGE];
    const int tid = threadIdx.x;
    const int col = tid % T2X;
    const int rg = tid / T2X;
    const double zinv = 1.0 / cf.z;
    const int nout = N;                      // node -> half lines: N+1 inputs, N outputs
    if (blockIdx.z == 0) {
        const int i0 = 1 + blockIdx.x * T2X;
        const int m0 = blockIdx.y * T2Y;
        if (i0 > N - 1 || m0 > N - 1) return;
        for (int e = tid; e < YH * T2X; e += NT2) {
            const int q = e / T2X, cc = e - q * T2X;
            const int i = i0 + cc, g = m0 - PADE_R + q;
            double v = 0.0;
            if (i <= N - 1 && g >= 0 && g <= N) v = ge_value<TRACKED>(src, g, i, N, P, cf.alpha);
            sg[e] = v;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < ROWS_PER_THREAD; ++t) {
            const int rr = rg + RG * t;
            const int m = m0 + rr, i = i0 + col;
            if (m < nout) {
                const double v = fir_any(L, taps, m, sg + rr * T2X + col, T2X);
                if (i <= N - 1) bx[(size_t)m * P + i] = -zinv * v;
            }
        }
    } else {
        const int m0 = blockIdx.x * T2X;
        const int j0 = 1 + blockIdx.y * T2Y;
        if (m0 > N - 1 || j0 > N - 1) return;
        for (int e = tid; e < T2Y * XW; e += NT2) {
            const int rr = e / XW, q = e - rr * XW;
            const int j = j0 + rr, g = m0 - PADE_R + q;
            double v = 0.0;
            if (j <= N - 1 && g >= 0 && g <= N) v = ge_value<TRACKED>(src, j, g, N, P, cf.alpha);
            sg[e] = v;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < ROWS_PER_THREAD; ++t) {
            const int rr = rg + RG * t;
            const int m = m0 + col, j = j0 + rr;
            if (m < nout) {
                const double v = fir_any(L, taps, m, sg + rr * XW + col, 1);
                if (j <= N - 1) by[(size_t)j * P + m] = zinv * v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Chebyshev solve of M Phi = b on one component grid, fused with the field
// update.  M = alpha I - beta L9, L9 = (1/6)[1 4 1; 4 -20 4; 1 4 1].  A tile
// of T2X x T2Y outputs is iterated in LDS together with a halo of K cells
// (one cell of the halo becomes invalid per application of M), so the solve
// reads b once and needs no global reduction.
// Boundaries: Dirichlet neighbours beyond the unknown range are zero; the
// Neumann ghost one cell beyond a half axis holds the mirrored value, which
// the owner of the boundary cell writes next to its own value.
// KIND 0: Ez with carried Laplacian, 1: Ez discrete, 2: Hx (z=0) / Hy (z=1).
// ---------------------------------------------------------------------------
struct ChebIO {
    const double* b;
    double* field;
    UGrid g;
};

template <int K, int KIND>
__global__ __launch_bounds__(NT2) void k_cheb_2d(ChebIO io0, ChebIO io1, double* __restrict__ ge,
                                                  const double* __restrict__ cur, int P, Coef cf,
                                                  ChebSchedule cs)
{
    constexpr int LW = T2X + 2 * K + 2;
    constexpr int LH = T2Y + 2 * K + 2;
    constexpr int IW = T2X + 2 * K;
    constexpr int IH = T2Y + 2 * K;
    constexpr int CPT = (IW * IH + NT2 - 1) / NT2;
    __shared__ double sd[LW * LH];
    const ChebIO& io = (KIND == 2 && blockIdx.z == 1) ? io1 : io0;
    const UGrid& g = io.g;
    const int x0 = g.lo[0] + blockIdx.x * T2X;
    const int y0 = g.lo[1] + blockIdx.y * T2Y;
    if (x0 >= g.hi[0] || y0 >= g.hi[1]) return;
    const int tid = threadIdx.x;
    for (int e = tid; e < LW * LH; e += NT2) sd[e] = 0.0;
    __syncthreads();

    double xv[CPT], rv[CPT], dv[CPT];
    int pos[CPT];        // LDS index of the cell, -1 when inactive
    int mir[CPT][3];     // LDS indices of mirror ghosts, -1 when none
    const double a = cf.alpha, bb = cf.beta * (1.0 / 6.0);
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int e = tid + q * NT2;
        pos[q] = -1;
        mir[q][0] = mir[q][1] = mir[q][2] = -1;
        xv[q] = rv[q] = dv[q] = 0.0;
        if (e < IW * IH) {
            const int iy = e / IW, ix = e - iy * IW;
            const int gx = x0 - K + ix, gy = y0 - K + iy;
            if (gx >= g.lo[0] && gx < g.hi[0] && gy >= g.lo[1] && gy < g.hi[1]) {
                const int p = (iy + 1) * LW + (ix + 1);
                pos[q] = p;
                const double r0 = io.b[(size_t)gy * P + gx];
                rv[q] = r0;
                dv[q] = r0 * cs.inv_theta;
                int mx = 0, my = 0;
                if (g.neumann[0]) mx = (gx == g.lo[0]) ? -1 : (gx == g.hi[0] - 1 ? 1 : 0);
                if (g.neumann[1]) my = (gy == g.lo[1]) ? -1 : (gy == g.hi[1] - 1 ? 1 : 0);
                if (mx) mir[q][0] = p + mx;
                if (my) mir[q][1] = p + my * LW;
                if (mx && my) mir[q][2] = p + mx + my * LW;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < CPT; ++q)
        if (pos[q] >= 0) {
            sd[pos[q]] = dv[q];
            for (int t = 0; t < 3; ++t)
                if (mir[q][t] >= 0) sd[mir[q][t]] = dv[q];
        }
    __syncthreads();

    for (int k = 0; k < K; ++k) {
        double ad[CPT];
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            ad[q] = 0.0;
            if (pos[q] >= 0) {
                const double* s = sd + pos[q];
                const double edge = s[-1] + s[1] + s[-LW] + s[LW];
                const double corner = s[-LW - 1] + s[-LW + 1] + s[LW - 1] + s[LW + 1];
                const double l9 = corner + 4.0 * edge - 20.0 * s[0];
                ad[q] = fma(a, s[0], -bb * l9);
            }
        }
        __syncthreads();
        const double c1 = cs.c1[k], c2 = cs.c2[k];
#pragma unroll
        for (int q = 0; q < CPT; ++q)
            if (pos[q] >= 0) {
                xv[q] += dv[q];
                rv[q] -= ad[q];
                dv[q] = fma(c1, dv[q], c2 * rv[q]);
                sd[pos[q]] = dv[q];
                for (int t = 0; t < 3; ++t)
                    if (mir[q][t] >= 0) sd[mir[q][t]] = dv[q];
            }
        __syncthreads();
    }

    // field update on the tile
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int e = tid + q * NT2;
        if (pos[q] < 0) continue;
        const int iy = e / IW, ix = e - iy * IW;
        if (ix < K || ix >= K + T2X || iy < K || iy >= K + T2Y) continue;
        const int gx = x0 - K + ix, gy = y0 - K + iy;
        const size_t o = (size_t)gy * P + gx;
        const double phi = xv[q] + dv[q];
        const double de = cf.cfl * phi;
        io.field[o] += de;
        if (KIND == 0) ge[o] += fma(cf.ge_gain, de, -cf.ge_curl * cur[o]);
    }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <int KIND>
static hipError_t launch_cheb_k(int K, dim3 grid, hipStream_t st, ChebIO io0, ChebIO io1, double* ge,
                                const double* cur, int P, Coef cf, ChebSchedule cs)
{
    switch (K) {
#define C4M_CASE(KK)                                                                              \
    case KK:                                                                                      \
        hipLaunchKernelGGL((k_cheb_2d<KK, KIND>), grid, dim3(NT2), 0, st, io0, io1, ge, cur, P, cf, \
                           cs);                                                                   \
        break;
        C4M_CASE(1) C4M_CASE(2) C4M_CASE(3) C4M_CASE(4) C4M_CASE(5) C4M_CASE(6) C4M_CASE(7) C4M_CASE(8)
#undef C4M_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_rhs_e_2d(hipStream_t st, bool tracked, const double* hx, const double* hy, double* t0,
                           double* t1, int N, int P, const Coef& cf, const PadeTaps& taps,
                           const PadeLine& line_h2n)
{
    dim3 grid((N - 1 + T2X - 1) / T2X, (N - 1 + T2Y - 1) / T2Y);
    if (tracked)
        hipLaunchKernelGGL(k_rhs_e2d<true>, grid, dim3(NT2), 0, st, hx, hy, t0, t1, N, P, cf, taps,
                           line_h2n);
    else
        hipLaunchKernelGGL(k_rhs_e2d<false>, grid, dim3(NT2), 0, st, hx, hy, t0, t1, N, P, cf, taps,
                           line_h2n);
    return hipGetLastError();
}

hipError_t launch_solve_e_2d(hipStream_t st, bool tracked, double* ez, double* ge, const double* t0,
                             const double* t1, int N, int P, const Coef& cf, const ChebSchedule& cs)
{
    dim3 grid((N - 1 + T2X - 1) / T2X, (N - 1 + T2Y - 1) / T2Y);
    ChebIO io{t0, ez, UGrid{{1, 1, 0}, {N, N, 1}, {0, 0, 0}}};
    if (tracked) return launch_cheb_k<0>(cs.sweeps, grid, st, io, io, ge, t1, P, cf, cs);
    return launch_cheb_k<1>(cs.sweeps, grid, st, io, io, nullptr, nullptr, P, cf, cs);
}

hipError_t launch_rhs_h_2d(hipStream_t st, bool tracked, const double* src, double* t0, double* t1,
                           int N, int P, const Coef& cf, const PadeTaps& taps,
                           const PadeLine& line_n2h)
{
    dim3 grid((N + T2X - 1) / T2X, (N + T2Y - 1) / T2Y, 2);
    if (tracked)
        hipLaunchKernelGGL(k_rhs_h2d<true>, grid, dim3(NT2), 0, st, src, t0, t1, N, P, cf, taps,
                           line_n2h);
    else
        hipLaunchKernelGGL(k_rhs_h2d<false>, grid, dim3(NT2), 0, st, src, t0, t1, N, P, cf, taps,
                           line_n2h);
    return hipGetLastError();
}

hipError_t launch_solve_h_2d(hipStream_t st, double* hx, double* hy, const double* t0,
                             const double* t1, int N, int P, const Coef& cf, const ChebSchedule& cs)
{
    dim3 grid((N + T2X - 1) / T2X, (N + T2Y - 1) / T2Y, 2);
    // Hx: Dirichlet in x (nodes 1..N-1), Neumann in y (half points 0..N-1)
    ChebIO iox{t0, hx, UGrid{{1, 0, 0}, {N, N, 1}, {0, 1, 0}}};
    // Hy: Neumann in x, Dirichlet in y
    ChebIO ioy{t1, hy, UGrid{{0, 1, 0}, {N, N, 1}, {1, 0, 0}}};
    return launch_cheb_k<2>(cs.sweeps, grid, st, iox, ioy, nullptr, nullptr, P, cf, cs);
}

}  // namespace c4m
