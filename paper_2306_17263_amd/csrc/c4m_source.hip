// c4m_source.hip -- the 2D (TM) step with a current J = (0, 0, Jz)
// (Section 3.1: eq:mh, Table tab:spec; Section 3.3: ghost values by Method 2,
// eq:gst2).
//
// The sourced step is the step without sources plus a correction, since
// every source term enters the right-hand side of a half-step linearly:
//   M Phi = b_0 + b_J,  Phi = M^{-1} b_0 + M^{-1} b_J,
// with b_0 the right-hand side of the step without sources (homogeneous
// ghosts) and b_J the rest:
//   Step 1 (Ez):  h (alpha F_J + h^2 Delta F_J / 12),  F_J = -Z (Jz + (h_t^2/24) Jz_tt),
//                 plus Z curl^A of the change of G(H) that the inhomogeneous H
//                 ghosts make at the first and last point of each H line;
//   Step 2 (H):   h (alpha F_J + h^2 Delta F_J / 12),  F_J = (h_t^2/24) curl dJ/dt,
//                 plus -(1/Z) curl^A of G_E on the E walls (h^2 Z dJz/dt / 12
//                 there: Delta Ez = Z dJz/dt where Ez vanishes), plus the
//                 inhomogeneous part of the ghosts of Phi_H in the rows of M
//                 next to the walls.
// The correction Phi_J = M^{-1} b_J is the problem's Chebyshev iteration on
// M (the three-term recurrence, K applications), run in one launch per
// component: a workgroup owns a T x T tile of unknowns, forms b_J over the
// tile and K points around it in LDS, applies M K times on shrinking
// windows (application k is valid k points inside the window), and adds r
// Phi_J to the field (and updates G_E with the carried Laplacian) on the
// tile.  The window is read from HBM once: the source arrays and the field.
//
// Scaling as in the rest of the library: Phi = h delta_t(field), curl^A the
// Pade curl without its 1/h, so the J terms enter multiplied by h.
#include "c4m_source.h"

namespace c4m {

// eq:gst2: the ghost offset along a half-point axis per unit h
__device__ __forceinline__ double ghost_q(const double* first, const double* third, int k, double h2_24)
{
    const double a = first ? first[k] : 0.0;
    const double c = third ? third[k] : 0.0;
    return fma(h2_24, c, a);
}

__device__ __forceinline__ double ld(const double* a, size_t k) { return a ? a[k] : 0.0; }

// Step 1 right-hand side b_J at the Ez unknown (i, j), 1 <= i, j <= N-1.
// wc: column 0 of A^{-1} for a half-to-node line (N - 1 values); by the
// reversal symmetry of the closure, its last column is wc read backwards.
__device__ double rhs_e_at(const SourceTM& s, const double* wc, int N, const SrcCoef& c, int i, int j)
{
    const size_t d = (size_t)j * (N + 1) + i;
    const double fj = -c.z * fma(c.ht2, ld(s.jz_tt, d), ld(s.jz, d));
    const double lj = -c.z * c.h * c.h * fma(c.ht2, ld(s.jz_tt_lap, d), ld(s.jz_lap, d));
    double v = c.h * fma(c.alpha, fj, lj * (1.0 / 12.0));
    // change of G(H) at the end points of the H lines: -h q_lo / 12 at the
    // first point, +h q_hi / 12 at the last; its Pade derivative at output
    // m is -W(m, 0) dg_lo + W(m, n-1) dg_hi  (n = N - 1 outputs).  W(m, 0)
    // decays like 0.0455^m: below 1e-32 W(0, 0) from PADE_B outputs on,
    // where the term is left out (the library's Pade rows stop there too).
    const int n = N - 1;
    if (i > PADE_B && i < n - PADE_B && j > PADE_B && j < n - PADE_B) return v;
    const double hx_lo = -c.h * ghost_q(s.hx_wall[0][0], s.hx_wall[0][1], i, c.h2_24) * (1.0 / 12.0);
    const double hx_hi = c.h * ghost_q(s.hx_wall[1][0], s.hx_wall[1][1], i, c.h2_24) * (1.0 / 12.0);
    const double hy_lo = -c.h * ghost_q(s.hy_wall[0][0], s.hy_wall[0][1], j, c.h2_24) * (1.0 / 12.0);
    const double hy_hi = c.h * ghost_q(s.hy_wall[1][0], s.hy_wall[1][1], j, c.h2_24) * (1.0 / 12.0);
    const int my = j - 1, mx = i - 1;
    const double dy = -wc[my] * hx_lo + wc[n - 1 - my] * hx_hi;   // d/dy of the change in G(Hx)
    const double dx = -wc[mx] * hy_lo + wc[n - 1 - mx] * hy_hi;   // d/dx of the change in G(Hy)
    return fma(c.z, dx - dy, v);
}

// inhomogeneous part of the Phi_H ghosts next to a half-point wall, moved to
// the right-hand side: beta (2/3 g(k) + 1/6 (g(k-1) + g(k+1))), g the ghost
// offset along the wall (zero at the node-wall ends, where Phi vanishes)
__device__ __forceinline__ double ghost_rows(const double* first, const double* third, int k, int N, double off,
                                             double h2_24, double beta)
{
    auto g = [&](int q) { return (q <= 0 || q >= N) ? 0.0 : off * ghost_q(first, third, q, h2_24); };
    return beta * ((2.0 / 3.0) * g(k) + (1.0 / 6.0) * (g(k - 1) + g(k + 1)));
}

// Step 2 right-hand side b_J at the unknown (i, j) of Hx (comp 0: x nodes
// 1..N-1, y half points 0..N-1) or Hy (comp 1: x half points, y nodes).
// vc: column 0 of A^{-1} for a node-to-half line (N values).
__device__ double rhs_h_at(const SourceTM& s, const double* vc, int comp, int N, const SrcCoef& c, int i, int j)
{
    const size_t d = comp == 0 ? (size_t)j * (N + 1) + i : (size_t)j * N + i;
    const double fj = c.ht2 * ld(comp == 0 ? s.kx : s.ky, d);
    const double lj = c.h * c.h * c.ht2 * ld(comp == 0 ? s.kx_lap : s.ky_lap, d);
    double v = c.h * fma(c.alpha, fj, lj * (1.0 / 12.0));
    // G_E on the two E walls the line crosses: h^2 Z dJz/dt / 12
    const double g12 = c.h * c.h * c.z * (1.0 / 12.0);
    const double h2 = c.h * c.h;
    const int n = N;   // outputs of a node-to-half line
    const int m = comp == 0 ? j : i;   // position along the derivative line (see rhs_e_at)
    if (m > PADE_B && m < n - 1 - PADE_B) return v;
    if (comp == 0) {   // -(1/Z) d/dy G_E along x = i
        const double lo = g12 * ld(s.jz_t, (size_t)i), hi = g12 * ld(s.jz_t, (size_t)N * (N + 1) + i);
        v -= (-vc[j] * lo + vc[n - 1 - j] * hi) / c.z;
        if (j == 0) v += ghost_rows(s.dhx_wall[0][0], s.dhx_wall[0][1], i, N, -h2, c.h2_24, c.beta);
        if (j == N - 1) v += ghost_rows(s.dhx_wall[1][0], s.dhx_wall[1][1], i, N, h2, c.h2_24, c.beta);
    } else {           // +(1/Z) d/dx G_E along y = j
        const double lo = g12 * ld(s.jz_t, (size_t)j * (N + 1)), hi = g12 * ld(s.jz_t, (size_t)j * (N + 1) + N);
        v += (-vc[i] * lo + vc[n - 1 - i] * hi) / c.z;
        if (i == 0) v += ghost_rows(s.dhy_wall[0][0], s.dhy_wall[0][1], j, N, -h2, c.h2_24, c.beta);
        if (i == N - 1) v += ghost_rows(s.dhy_wall[1][0], s.dhy_wall[1][1], j, N, h2, c.h2_24, c.beta);
    }
    return v;
}

// One component's correction on a T x T tile (see the top of the file).
// Window: W = T + 2K points per side around the tile, in storage indices
// from (rx, ry), holding b and two iterates.  Application k (1..K) of the
// first-order Chebyshev form (the residual polynomial of the three-term
// recurrence with the same K applications, no x_{k-1} read)
//   x_{k+1} = x_k + w_k (b - M x_k),  x_1 = w_0 b,
// runs on window points k .. W-1-k; x_{k+1} goes to buf[(k+1) % 2], the last
// one into the field.
// M = alpha I - beta L9 with the homogeneous wall rules is a plain 9-point
// stencil on the window because the window holds them explicitly: zero on
// the node walls (never written), and at the first point beyond a half-axis
// wall the value of its mirror image (written with it).  Points further out
// are never read.
template <int T, int NT>
__global__ __launch_bounds__(NT) void k_src_tile(SrcTile a)
{
    static_assert(T + 2 * MAX_SWEEPS <= 64, "a window row must fit one wave");
    extern __shared__ double lds[];
    const ChebGeom& g = a.g;
    const int K = a.K, W = T + 2 * K, WW = W * W;
    double* sb = lds;
    double* buf[2] = {lds + WW, lds + 2 * WW};
    const int rx = g.lo[0] + (int)blockIdx.x * T - K;
    const int ry = g.lo[1] + (int)blockIdx.y * T - K;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    constexpr int RS = NT / 64;
    // storage index of the image of window point (li, lj) under the wall
    // rules, or false (a node wall or further out: zero / never read)
    auto image = [&](int li, int lj, int& i, int& j) -> bool {
        i = rx + li;
        j = ry + lj;
        if (g.half[0]) i = i == -1 ? 0 : (i == g.n[0] ? g.n[0] - 1 : i);
        if (g.half[1]) j = j == -1 ? 0 : (j == g.n[1] ? g.n[1] - 1 : j);
        return i >= g.lo[0] && i <= g.hi[0] && j >= g.lo[1] && j <= g.hi[1];
    };
    if (tx < W) {
#pragma unroll 4
        for (int lj = ty; lj < W; lj += RS) {
            const int q = lj * W + tx;
            int i, j;
            double v = 0.0;
            if (image(tx, lj, i, j))
                v = a.comp == 2 ? rhs_e_at(a.s, a.cols, a.N, a.c, i, j) : rhs_h_at(a.s, a.cols, a.comp, a.N, a.c, i, j);
            sb[q] = v;
            buf[0][q] = 0.0;
            buf[1][q] = 0.0;
        }
    }
    __syncthreads();
    // Each thread owns window column li and a run of consecutive rows and
    // marches down them with the 3 x 3 neighbourhood in registers (three
    // new LDS values per point).  A point next to a half-axis wall also
    // writes its value to its mirror ghost.
    const bool half_x = g.half[0] != 0, half_y = g.half[1] != 0;
    for (int k = 1; k <= K; ++k) {
        const double* xk = k == 1 ? sb : buf[k % 2];
        const double sc = k == 1 ? a.w[0] : 1.0;
        double* out = buf[(k + 1) % 2];
        const double wk = a.w[k];
        const int span = W - 2 * k;
        const int run = (span + RS - 1) / RS;
        const int li = k + tx;
        const int j0 = k + ty * run, j1 = min(j0 + run, W - k);
        if (tx < span && j0 < j1) {
            const int i = rx + li;
            const bool col_in = i >= g.lo[0] && i <= g.hi[0];
            const double* c0 = xk + li;
            double a0 = c0[(j0 - 1) * W - 1], a1 = c0[(j0 - 1) * W], a2 = c0[(j0 - 1) * W + 1];
            double b0 = c0[j0 * W - 1], b1 = c0[j0 * W], b2 = c0[j0 * W + 1];
            for (int lj = j0; lj < j1; ++lj) {
                const double d0 = c0[(lj + 1) * W - 1], d1 = c0[(lj + 1) * W], d2 = c0[(lj + 1) * W + 1];
                const int j = ry + lj;
                if (col_in && j >= g.lo[1] && j <= g.hi[1]) {
                    const double xc = b1 * sc;
                    const double faces = (b0 + b2 + a1 + d1) * sc;
                    const double corners = (a0 + a2 + d0 + d2) * sc;
                    const double l9 = (2.0 / 3.0) * faces + (1.0 / 6.0) * corners - (10.0 / 3.0) * xc;
                    const int wp = lj * W + li;
                    const double bo = sb[wp];
                    const double mx = fma(g.alpha, xc, -g.beta * l9);
                    const double xn = fma(wk, bo - mx, xc);
                    if (k < K) {
                        out[wp] = xn;
                        // mirror ghosts (first point beyond a half-axis wall)
                        const int ex = half_x ? (i == 0 ? -1 : (i == g.n[0] - 1 ? 1 : 0)) : 0;
                        const int ey = half_y ? (j == 0 ? -W : (j == g.n[1] - 1 ? W : 0)) : 0;
                        if (ex) out[wp + ex] = xn;
                        if (ey) out[wp + ey] = xn;
                        if (ex && ey) out[wp + ex + ey] = xn;
                    } else if (lj >= K && lj < K + T && li >= K && li < K + T) {
                        // the last application: the tile's points update the field
                        const size_t o = (size_t)j * g.P + i;
                        const double de = a.u.r * xn;
                        a.u.field[o] += de;
                        if (a.u.ge) {   // G_E += (1 + 4/r^2) dE - (2/r) h F_J   (the carried Laplacian)
                            const size_t d = (size_t)j * g.n[0] + i;
                            const double fj = -a.u.z * fma(a.u.ht2, ld(a.u.jz_tt, d), ld(a.u.jz, d));
                            a.u.ge[o] += fma(a.u.ge_gain, de, -a.u.ge_src * fj);
                        }
                    }
                }
                a0 = b0; a1 = b1; a2 = b2;
                b0 = d0; b1 = d1; b2 = d2;
            }
        }
        if (k < K) __syncthreads();
    }
}

constexpr int SRC_TILE = 48, SRC_THREADS = 512;

size_t src_tile_lds(int K)
{
    const size_t w = SRC_TILE + 2 * (size_t)K;
    return 3 * w * w * sizeof(double);
}

hipError_t launch_src_group(hipStream_t st, const SrcTile& a0)
{
    if (a0.K < 1 || a0.K > MAX_SWEEPS) return hipErrorInvalidValue;
    // w_j = 1 / mu_j at the K + 1 Chebyshev roots on [alpha, alpha + 16 beta / 3]
    SrcTile a = a0;
    const double lmin = a.g.alpha, lmax = a.g.alpha + 16.0 / 3.0 * a.g.beta;
    for (int j = 0; j <= a.K; ++j)
        a.w[j] = 1.0 / (0.5 * (lmax + lmin) - 0.5 * (lmax - lmin) * cos((2 * j + 1) * M_PI / (2.0 * (a.K + 1))));
    const int nx = a.g.hi[0] - a.g.lo[0] + 1, ny = a.g.hi[1] - a.g.lo[1] + 1;
    const dim3 grid((unsigned)((nx + SRC_TILE - 1) / SRC_TILE), (unsigned)((ny + SRC_TILE - 1) / SRC_TILE));
    hipLaunchKernelGGL((k_src_tile<SRC_TILE, SRC_THREADS>), grid, dim3(SRC_THREADS), src_tile_lds(a.K), st, a);
    return hipGetLastError();
}

}  // namespace c4m
