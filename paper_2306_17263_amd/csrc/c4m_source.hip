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
// The correction Phi_J = M^{-1} b_J runs as a plain Chebyshev iteration on M
// (the schedule of the problem), one launch per application of M; its last
// launch updates the field (and G_E with the carried Laplacian).
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

// Step 1 right-hand side b_J at the Ez unknowns (x, y = 1..N-1).
// wc: column 0 of A^{-1} for a half-to-node line (N - 1 values); by the
// reversal symmetry of the closure, its last column is wc read backwards.
__global__ void k_src_rhs_e(double* b, SourceTM s, const double* wc, int N, int P, SrcCoef c)
{
    const int i = 1 + blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = 1 + blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i > N - 1 || j > N - 1) return;
    const size_t d = (size_t)j * (N + 1) + i;
    const double fj = -c.z * fma(c.ht2, ld(s.jz_tt, d), ld(s.jz, d));
    const double lj = -c.z * c.h * c.h * fma(c.ht2, ld(s.jz_tt_lap, d), ld(s.jz_lap, d));
    double v = c.h * fma(c.alpha, fj, lj * (1.0 / 12.0));
    // change of G(H) at the end points of the H lines: -h q_lo / 12 at the
    // first point, +h q_hi / 12 at the last; its Pade derivative at output
    // m is -W(m, 0) dg_lo + W(m, n-1) dg_hi  (n = N - 1 outputs)
    const int n = N - 1;
    const double hx_lo = -c.h * ghost_q(s.hx_wall[0][0], s.hx_wall[0][1], i, c.h2_24) * (1.0 / 12.0);
    const double hx_hi = c.h * ghost_q(s.hx_wall[1][0], s.hx_wall[1][1], i, c.h2_24) * (1.0 / 12.0);
    const double hy_lo = -c.h * ghost_q(s.hy_wall[0][0], s.hy_wall[0][1], j, c.h2_24) * (1.0 / 12.0);
    const double hy_hi = c.h * ghost_q(s.hy_wall[1][0], s.hy_wall[1][1], j, c.h2_24) * (1.0 / 12.0);
    const int my = j - 1, mx = i - 1;
    const double dy = -wc[my] * hx_lo + wc[n - 1 - my] * hx_hi;   // d/dy of the change in G(Hx)
    const double dx = -wc[mx] * hy_lo + wc[n - 1 - mx] * hy_hi;   // d/dx of the change in G(Hy)
    v += c.z * (dx - dy);
    b[(size_t)j * P + i] = v;
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

// Step 2 right-hand side b_J of Hx (comp 0: x nodes 1..N-1, y half points
// 0..N-1) or Hy (comp 1: x half points 0..N-1, y nodes 1..N-1).
// vc: column 0 of A^{-1} for a node-to-half line (N values).
__global__ void k_src_rhs_h(double* b, SourceTM s, const double* vc, int comp, int N, int P, SrcCoef c)
{
    const int a = blockIdx.x * 64 + (threadIdx.x & 63);       // x
    const int t = blockIdx.y * 4 + (threadIdx.x >> 6);        // y
    const int i = comp == 0 ? a + 1 : a;
    const int j = comp == 0 ? t : t + 1;
    if (i > N - 1 || j > N - 1) return;
    const size_t d = comp == 0 ? (size_t)j * (N + 1) + i : (size_t)j * N + i;
    const double* k = comp == 0 ? s.kx : s.ky;
    const double* kl = comp == 0 ? s.kx_lap : s.ky_lap;
    const double fj = c.ht2 * ld(k, d);
    const double lj = c.h * c.h * c.ht2 * ld(kl, d);
    double v = c.h * fma(c.alpha, fj, lj * (1.0 / 12.0));
    // G_E on the two E walls the line crosses: h^2 Z dJz/dt / 12
    const double g12 = c.h * c.h * c.z * (1.0 / 12.0);
    const int n = N;   // outputs of a node-to-half line
    if (comp == 0) {   // -(1/Z) d/dy G_E along x = i
        const double lo = g12 * ld(s.jz_t, (size_t)i), hi = g12 * ld(s.jz_t, (size_t)N * (N + 1) + i);
        v -= (-vc[j] * lo + vc[n - 1 - j] * hi) / c.z;
        const double h2 = c.h * c.h;
        if (j == 0) v += ghost_rows(s.dhx_wall[0][0], s.dhx_wall[0][1], i, N, -h2, c.h2_24, c.beta);
        if (j == N - 1) v += ghost_rows(s.dhx_wall[1][0], s.dhx_wall[1][1], i, N, h2, c.h2_24, c.beta);
    } else {           // +(1/Z) d/dx G_E along y = j
        const double lo = g12 * ld(s.jz_t, (size_t)j * (N + 1)), hi = g12 * ld(s.jz_t, (size_t)j * (N + 1) + N);
        v += (-vc[i] * lo + vc[n - 1 - i] * hi) / c.z;
        const double h2 = c.h * c.h;
        if (i == 0) v += ghost_rows(s.dhy_wall[0][0], s.dhy_wall[0][1], j, N, -h2, c.h2_24, c.beta);
        if (i == N - 1) v += ghost_rows(s.dhy_wall[1][0], s.dhy_wall[1][1], j, N, h2, c.h2_24, c.beta);
    }
    b[(size_t)j * P + i] = v;
}

// One application of M in the three-term Chebyshev recurrence
//   x_{k+1} = x_k + c1 (x_k - x_{k-1}) + c2 (b - M x_k),  x_0 = 0, x_1 = b / theta,
// M = alpha I - beta L9 with homogeneous walls: zero beyond a node axis'
// unknowns, even ghosts along a half axis.  cur: 0 = x_k is b / theta,
// 1 = x_k in xk.  prev: 0 = x_{k-1} is 0, 1 = b / theta, 2 = in out.
// x_{k+1} goes to out (over x_{k-1}, read at the same point first) or, on
// the last application, into the field update.
__global__ void k_src_cheb(const double* b, const double* xk, double* out, ChebGeom g, double c1, double c2,
                           int cur, int prev, SrcUpdate u)
{
    const int i = g.lo[0] + blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = g.lo[1] + blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i > g.hi[0] || j > g.hi[1]) return;
    const int P = g.P;
    auto val = [&](int x, int y) -> double {
        if (g.half[0]) x = x < 0 ? -1 - x : (x >= g.n[0] ? 2 * g.n[0] - 1 - x : x);
        else if (x <= 0 || x >= g.n[0] - 1) return 0.0;
        if (g.half[1]) y = y < 0 ? -1 - y : (y >= g.n[1] ? 2 * g.n[1] - 1 - y : y);
        else if (y <= 0 || y >= g.n[1] - 1) return 0.0;
        const size_t o = (size_t)y * P + x;
        return cur == 0 ? b[o] * g.inv_theta : xk[o];
    };
    const size_t o = (size_t)j * P + i;
    const double xc = val(i, j);
    const double faces = val(i - 1, j) + val(i + 1, j) + val(i, j - 1) + val(i, j + 1);
    const double corners = val(i - 1, j - 1) + val(i + 1, j - 1) + val(i - 1, j + 1) + val(i + 1, j + 1);
    const double l9 = (2.0 / 3.0) * faces + (1.0 / 6.0) * corners - (10.0 / 3.0) * xc;
    const double bo = b[o];
    const double mx = fma(g.alpha, xc, -g.beta * l9);
    const double xp = prev == 0 ? 0.0 : (prev == 1 ? bo * g.inv_theta : out[o]);
    const double xn = xc + c1 * (xc - xp) + c2 * (bo - mx);
    if (!u.field) {
        out[o] = xn;
        return;
    }
    const double de = u.r * xn;
    u.field[o] += de;
    if (u.ge) {   // G_E += (1 + 4/r^2) dE - (2/r) h F_J   (the carried Laplacian)
        const size_t d = (size_t)j * (g.n[0]) + i;
        const double fj = -u.z * fma(u.ht2, ld(u.jz_tt, d), ld(u.jz, d));
        u.ge[o] += fma(u.ge_gain, de, -u.ge_src * fj);
    }
}

namespace {
inline dim3 grid_of(int nx, int ny) { return dim3((unsigned)((nx + 63) / 64), (unsigned)((ny + 3) / 4)); }
}  // namespace

hipError_t launch_src_rhs_e(hipStream_t st, double* b, const SourceTM& s, const double* wc, int N, int P,
                            const SrcCoef& c)
{
    hipLaunchKernelGGL(k_src_rhs_e, grid_of(N - 1, N - 1), dim3(256), 0, st, b, s, wc, N, P, c);
    return hipGetLastError();
}

hipError_t launch_src_rhs_h(hipStream_t st, double* b, const SourceTM& s, const double* vc, int comp, int N,
                            int P, const SrcCoef& c)
{
    const int nx = comp == 0 ? N - 1 : N, ny = comp == 0 ? N : N - 1;
    hipLaunchKernelGGL(k_src_rhs_h, grid_of(nx, ny), dim3(256), 0, st, b, s, vc, comp, N, P, c);
    return hipGetLastError();
}

hipError_t launch_src_solve(hipStream_t st, const double* b, double* xa, double* xb, const ChebGeom& g,
                            const ChebSchedule& cs, const SrcUpdate& u)
{
    const dim3 grid = grid_of(g.hi[0] - g.lo[0] + 1, g.hi[1] - g.lo[1] + 1);
    const SrcUpdate none{};
    // application k = 1..K reads x_k and x_{k-1}, writes x_{k+1}:
    // x_2 -> xa, x_3 -> xb, x_4 -> xa (over x_2), ...
    double* buf[2] = {xa, xb};
    const int K = cs.sweeps;
    for (int k = 1; k <= K; ++k) {
        const int cur = k == 1 ? 0 : 1;
        const int prev = k == 1 ? 0 : (k == 2 ? 1 : 2);
        const double* xk = k == 1 ? nullptr : buf[k % 2];          // x_k written by application k-1
        double* out = buf[(k + 1) % 2];                              // holds x_{k-1} for k >= 3
        hipLaunchKernelGGL(k_src_cheb, grid, dim3(256), 0, st, b, xk, out, g, cs.c1[k - 1], cs.c2[k - 1], cur,
                           prev, k == K ? u : none);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace c4m
