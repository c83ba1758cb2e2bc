// c4m_kernels_3d.hip -- gfx950 kernels of the full 3D step (Ex..Hz).
//
// Step 1 (Section 3.4): the conditioned sources G(H_j) once (k_condition3),
// then per E component s (s1 = s+1, s2 = s+2 mod 3):
//   b   = Z (delta_{s1} G(H_{s2}) - delta_{s2} G(H_{s1}))      two line terms
//   c   = delta_{s1} H_{s2} - delta_{s2} H_{s1}                 (carried l) two more
//   Phi = M^{-1} b (19-point M), E_s += r Phi, G_E += ...       K Chebyshev passes
// Step 2, per H component s:
//   b   = -(1/Z) (delta_{s1} G_{E,s2} - delta_{s2} G_{E,s1}),   H_s += r M^{-1} b
// (G_E stored, or G(E_j) conditioned once for the discrete Laplacian).
//
// Line terms: along x, k_term3 stages the line windows of a tile in LDS
// (coalesced loads) and runs the truncated Pade FIR over a register window
// of 8 outputs per thread; along y and z, k_march3 streams each wave along
// its lines with a register window.  Chebyshev: three-term form, one
// z-marching launch per application of M with the planes of the iterate in
// an LDS ring (k_cheb3t); the FP32-refined form runs the same passes with
// FP32 iterates around one FP64 residual.  The FP64 Chebyshev step is
// recorded as a list of launches (plan_step3) that a single problem replays
// and a batch runs over all its members (the *_b kernels).
#include <string.h>

#include "c4m_internal.h"

namespace c4m {

enum { SRC_RAW = 0, SRC_G = 1, SRC_GE_STORED = 2, SRC_GE_DISCRETE = 3 };


__device__ __forceinline__ const double* pade_row3(const PadeLine& L, int m)
{
    if (L.all) return L.rows + (size_t)m * PADE_TAPS;
    if (m < L.b) return L.rows + (size_t)m * PADE_TAPS;
    if (m >= L.n_out - L.b) return L.rows + (size_t)(m - (L.n_out - L.b) + L.b) * PADE_TAPS;
    return L.rows + (size_t)(2 * L.b) * PADE_TAPS;   // the interior taps, stored after the boundary rows
}

// Source value at stored index q (q[D] may run outside the line: zero; ok
// false: zero).  SRC_G: alpha u + (sum of second differences)/12 with even
// ghosts along half axes (node axes are interior here); SRC_GE_DISCRETE: the
// same on E, zero on E's node walls.  Every load takes an index clamped into
// the stored box and the value is selected at the end, so a caller can have
// the loads of several values in flight at once.
template <int MODE>
__device__ __forceinline__ double src_value(const Term3& t, int i, int j, int k, double alpha, bool ok, double& raw)
{
    const Box& b = t.sb;
    const int q[3] = {i, j, k};
    int c[3];
    bool in = ok;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        in = in && q[d] >= 0 && q[d] < b.n[d];
        c[d] = q[d] < 0 ? 0 : (q[d] >= b.n[d] ? b.n[d] - 1 : q[d]);
    }
    const double* p = t.src + c[2] * t.plane + (size_t)c[1] * t.P + c[0];
    const double u0 = p[0];
    raw = in ? u0 : 0.0;
    if (MODE == SRC_RAW || MODE == SRC_GE_STORED) return raw;
    const long st[3] = {1, (long)t.P, (long)t.plane};
    if (MODE == SRC_GE_DISCRETE) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
            if (!b.half[d]) in = in && c[d] != 0 && c[d] != b.n[d] - 1;
    }
    double lap = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double um = p[c[d] == 0 ? 0 : -st[d]];                 // even ghost (half axis)
        const double up = p[c[d] == b.n[d] - 1 ? 0 : st[d]];
        lap += um + up - 2.0 * u0;
    }
    return in ? fma(alpha, u0, lap * (1.0 / 12.0)) : 0.0;
}

constexpr int T3_SEG = 8;

// LDS doubles of a k_term3 tile along axis D
template <int D>
constexpr int term3_lds()
{
    constexpr int A = D == 0 ? 32 : 64, NO = D == 0 ? 64 : 32, BW = NO + PADE_TAPS - 1;
    return A * ((BW % 2) ? BW : BW + 1);
}

// One tile (block coordinates blk) of the line term; sv: term3_lds<D>() doubles of LDS.
template <int D, int MODE>
__device__ __forceinline__ void term3_body(const Term3& t, double alpha, const PadeTaps& taps, const PadeLine& L,
                                           uint3 blk, double* sv)
{
    // tile geometry: A lines x NO outputs per line
    constexpr int A = D == 0 ? 32 : 64;
    constexpr int NO = D == 0 ? 64 : 32;
    constexpr int BW = NO + PADE_TAPS - 1;       // staged window per line
    constexpr int BS = (BW % 2) ? BW : BW + 1;   // odd stride
    // axes: D = line axis, W = across lines in the tile, Sx = slab (blockIdx.z)
    constexpr int W = D == 0 ? 1 : 0;
    constexpr int SX = 3 - D - W;
    const int m0 = blk.x * NO;                            // first output along D
    const int w0 = t.tg.lo[W] + blk.y * A;                // first line along W
    const int s = t.tg.lo[SX] + blk.z;                    // slab index
    const int tid = threadIdx.x;
    const int n_in = L.n_in;
    // staging in chunks of CH elements per thread, the loads of a chunk all
    // in flight before its LDS stores
    constexpr int NS = (A * BW + 255) / 256;
    constexpr int CH = (MODE == SRC_RAW || MODE == SRC_GE_STORED) ? NS : 4;
    for (int i0 = 0; i0 < NS; i0 += CH) {
        double v[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int e = tid + (i0 + c) * 256;
            int a, q;
            if (D == 0) { a = e / BW; q = e - a * BW; }   // consecutive threads along the line (x)
            else { q = e / A; a = e - q * A; }            // consecutive threads across lines (x)
            const int wi = w0 + a;
            const int g = m0 - PADE_R + q;
            const bool ok = i0 + c < NS && e < A * BW && wi < t.tg.hi[W] && g >= 0 && g < n_in;
            int idx[3];
            idx[D] = g;
            idx[W] = wi;
            idx[SX] = s;
            double raw;
            v[c] = src_value<MODE>(t, idx[0], idx[1], idx[2], alpha, ok, raw);
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int e = tid + (i0 + c) * 256;
            int a, q;
            if (D == 0) { a = e / BW; q = e - a * BW; }
            else { q = e / A; a = e - q * A; }
            if (i0 + c < NS && e < A * BW) sv[a * BS + q] = v[c];
        }
    }
    __syncthreads();
    // thread -> (line a, segment): lanes of a half-wave take consecutive lines
    const int a = tid % A;
    const int seg = tid / A;
    const int mb = m0 + seg * T3_SEG;
    const bool fast = !L.all && mb >= L.b && mb + T3_SEG - 1 < L.n_out - L.b;
    auto fir = [&](const double* w, double (&out)[T3_SEG]) {
        if (fast) {
            double win[T3_SEG + PADE_TAPS - 1];
#pragma unroll
            for (int u = 0; u < T3_SEG + PADE_TAPS - 1; ++u) win[u] = w[u];
#pragma unroll
            for (int k = 0; k < T3_SEG; ++k) {
                double acc = 0.0;
#pragma unroll
                for (int u = 0; u < PADE_TAPS; ++u) acc = fma(taps.c[u], win[k + u], acc);
                out[k] = acc;
            }
        } else {
#pragma unroll
            for (int k = 0; k < T3_SEG; ++k) {
                const int m = mb + k;
                double acc = 0.0;
                if (m < L.n_out) {
                    const double* cr = pade_row3(L, m);
                    for (int u = 0; u < PADE_TAPS; ++u) acc = fma(cr[u], w[k + u], acc);
                }
                out[k] = acc;
            }
        }
    };
    double out[T3_SEG];
    fir(sv + a * BS + seg * T3_SEG, out);
    if (D == 0) {
        // x-lines: a thread's outputs run along x, so store through the LDS
        // and let consecutive lanes write consecutive x positions
        constexpr int OS = NO + 1;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < T3_SEG; ++k) sv[a * OS + seg * T3_SEG + k] = out[k];
        __syncthreads();
        for (int e = tid; e < A * NO; e += 256) {
            const int la = e / NO, c = e - la * NO;
            const int wl = w0 + la, m = m0 + c;
            if (wl >= t.tg.hi[W] || m >= L.n_out) continue;
            const size_t oi = s * t.plane + (size_t)wl * t.P + (t.tg.lo[0] + m);
            const double v = t.scale * sv[la * OS + c];
            t.out[oi] = t.accumulate ? t.out[oi] + v : v;
        }
        return;
    }
    const int wi = w0 + a;
    if (wi >= t.tg.hi[W]) return;
#pragma unroll
    for (int k = 0; k < T3_SEG; ++k) {
        const int m = mb + k;
        if (m >= L.n_out) break;
        int idx[3];
        idx[D] = t.tg.lo[D] + m;
        idx[W] = wi;
        idx[SX] = s;
        const size_t oi = idx[2] * t.plane + (size_t)idx[1] * t.P + idx[0];
        const double v = t.scale * out[k];
        t.out[oi] = t.accumulate ? t.out[oi] + v : v;
    }
}

template <int D, int MODE>
__global__ __launch_bounds__(256) void k_term3(Term3 t, double alpha, PadeTaps taps, PadeLine L)
{
    __shared__ double sv[term3_lds<D>()];
    term3_body<D, MODE>(t, alpha, taps, L, make_uint3(blockIdx.x, blockIdx.y, blockIdx.z), sv);
}

// k_condition3: the conditioned source G(u) (SRC_G) or its discrete-
// Laplacian form on E (SRC_GE_DISCRETE) at every stored point of a box, as
// src_value forms it, so that the line terms can read it raw.
template <int MODE>
__device__ __forceinline__ void condition3_body(const Term3& t, double alpha, uint3 blk)
{
    // 64 x 4 points of a plane per workgroup (a row of 257 points leaves
    // one lane busy in its last block, not 255 idle)
    const int i = blk.x * 64 + (threadIdx.x & 63);
    const int j = blk.y * 4 + (threadIdx.x >> 6), k = blk.z;
    if (i >= t.sb.n[0] || j >= t.sb.n[1]) return;
    double raw;
    t.out[(size_t)k * t.plane + (size_t)j * t.P + i] = src_value<MODE>(t, i, j, k, alpha, true, raw);
}

template <int MODE>
__global__ __launch_bounds__(256) void k_condition3(Term3 t, double alpha)
{
    condition3_body<MODE>(t, alpha, make_uint3(blockIdx.x, blockIdx.y, blockIdx.z));
}

// k_march3: the same line term along y or z (D = 1, 2) as a streaming pass.
// A wave owns 64 consecutive x positions at one index of the third axis and
// marches along its lines over a segment of outputs; the conditioned inputs
// of the current block of Q outputs sit in a register window (Q + 25
// values), and the inputs of the next block are loaded before the current
// block's FIR runs, so their latency overlaps the arithmetic.  Taps and
// summation order are those of k_term3.
constexpr int M3_Q = 8, M3_WIN = M3_Q + PADE_TAPS - 1;

template <int D, int MODE>
__device__ __forceinline__ void march3_body(const Term3& t, double alpha, const PadeTaps& taps, const PadeLine& L,
                                            int seg_len, uint3 blk)
{
    constexpr int T = 3 - D;                       // third axis (x is always across lanes)
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
    const int xi = t.tg.lo[0] + blk.x * 64 + lane;
    const int ti = t.tg.lo[T] + blk.y * 4 + wv;
    if (xi >= t.tg.hi[0] || ti >= t.tg.hi[T]) return;
    const int m0 = blk.z * seg_len;
    const int m1 = min(m0 + seg_len, L.n_out);
    const int n_in = L.n_in;
    auto input = [&](int g) {
        int idx[3];
        idx[0] = xi;
        idx[D] = g;
        idx[T] = ti;
        double raw;
        return src_value<MODE>(t, idx[0], idx[1], idx[2], alpha, g >= 0 && g < n_in, raw);
    };
    double win[M3_WIN], nxt[M3_Q];
#pragma unroll
    for (int u = 0; u < PADE_TAPS - 1; ++u) win[u] = input(m0 - PADE_R + u);
#pragma unroll
    for (int q = 0; q < M3_Q; ++q) nxt[q] = input(m0 - PADE_R + PADE_TAPS - 1 + q);
    size_t o = (size_t)(D == 2 ? t.tg.lo[2] + m0 : ti) * t.plane + (size_t)(D == 1 ? t.tg.lo[1] + m0 : ti) * t.P + xi;
    const size_t ostep = D == 2 ? t.plane : (size_t)t.P;
    for (int mb = m0; mb < m1; mb += M3_Q) {
#pragma unroll
        for (int q = 0; q < M3_Q; ++q) win[PADE_TAPS - 1 + q] = nxt[q];
        // the accumulated outputs are read before the prefetch is issued
        // (loads complete in order, so a later read would wait for it)
        double prev[M3_Q];
#pragma unroll
        for (int k = 0; k < M3_Q; ++k)
            prev[k] = (t.accumulate && mb + k < m1) ? t.out[o + (size_t)k * ostep] : 0.0;
        if (mb + M3_Q < m1) {
#pragma unroll
            for (int q = 0; q < M3_Q; ++q) nxt[q] = input(mb + M3_Q - PADE_R + PADE_TAPS - 1 + q);
        }
        const bool fast = !L.all && mb >= L.b && mb + M3_Q - 1 < L.n_out - L.b;
#pragma unroll
        for (int k = 0; k < M3_Q; ++k) {
            const int m = mb + k;
            if (m >= m1) break;
            double acc = 0.0;
            if (fast) {
#pragma unroll
                for (int u = 0; u < PADE_TAPS; ++u) acc = fma(taps.c[u], win[k + u], acc);
            } else {
                const double* cr = pade_row3(L, m);
#pragma unroll
                for (int u = 0; u < PADE_TAPS; ++u) acc = fma(cr[u], win[k + u], acc);
            }
            const double v = t.scale * acc;
            t.out[o] = t.accumulate ? prev[k] + v : v;
            o += ostep;
        }
#pragma unroll
        for (int u = 0; u < PADE_TAPS - 1; ++u) win[u] = win[u + M3_Q];
    }
}

template <int D, int MODE>
__global__ __launch_bounds__(256) void k_march3(Term3 t, double alpha, PadeTaps taps, PadeLine L, int seg_len)
{
    march3_body<D, MODE>(t, alpha, taps, L, seg_len, make_uint3(blockIdx.x, blockIdx.y, blockIdx.z));
}

// ---------------------------------------------------------------------------
// Solve: Chebyshev in three-term form on the same schedule,
//   x_1 = b / theta,  x_{k+1} = x_k + c1_{k-1} (x_k - x_{k-1}) + c2_{k-1} (b - M x_k),
// k = 1..K, Phi = x_{K+1} (K applications of M).  Each application is one
// z-marching pass over the grid: a workgroup owns a 64 x 4 column tile and
// a chunk of planes, and keeps the three planes z-1, z, z+1 of x_k (with a
// one-point ring, boundary rules applied when loading) in a 4-deep LDS ring.
// The first pass reads only b; the last writes the field update.
//
// The FP32-refined form runs the same passes with FP32 iterates: a round
// x1 = C(b) of s applications, one FP64 pass forming res = b - M x1, and a
// round x2 = C(res) whose last pass writes field += cfl (x1 + x2).
// ---------------------------------------------------------------------------
constexpr int C3_TX = 64, C3_TY = 4, C3_CZ = 16;
constexpr int C3_LX = C3_TX + 2, C3_LY = C3_TY + 2, C3_PL = C3_LX * C3_LY;



// Index of grid point (i, j, k) after the boundary rules of the unknowns:
// Dirichlet outside the range -> -1 (zero), Neumann -> mirrored onto the
// edge unknown.
__device__ __forceinline__ long rule_index(const UGrid& g, int P, size_t plane, int i, int j, int k)
{
    int q[3] = {i, j, k};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (q[d] < g.lo[d]) {
            if (!g.neumann[d]) return -1;
            q[d] = g.lo[d];
        } else if (q[d] >= g.hi[d]) {
            if (!g.neumann[d]) return -1;
            q[d] = g.hi[d] - 1;
        }
    }
    return (long)q[2] * (long)plane + (long)q[1] * P + q[0];
}

// TC: arithmetic type of the pass; ring: 4 C3_PL planes of LDS.
template <class TX, class TB, class TC, bool FIRST, int OUT>
__device__ __forceinline__ void cheb3t_body(const Cheb3T<TX, TB>& a, uint3 blk, TC (*ring)[C3_PL])
{
    const int tid = threadIdx.x;
    const int tx = tid % C3_TX, ty = tid / C3_TX;
    const int bx = a.g.lo[0] + blk.x * C3_TX, by = a.g.lo[1] + blk.y * C3_TY;
    const int i = bx + tx, j = by + ty;
    const int z0 = a.g.lo[2] + blk.z * C3_CZ;
    const int z1 = min(z0 + C3_CZ, a.g.hi[2]);
    const bool own = i < a.g.hi[0] && j < a.g.hi[1];
    const TC scale = FIRST ? TC(a.inv_theta) : TC(1);
    // Planes of the iterate (with the halo) pass through registers into the
    // LDS ring: the loads of plane z + 2 are issued in the iteration of plane
    // z and stored to the ring in the next one.  Loads take clamped (valid)
    // indices and the value is selected after.
    constexpr int NL = (C3_PL + 255) / 256;
    auto fetch = [&](int z, TC (&r)[NL]) {
#pragma unroll
        for (int c = 0; c < NL; ++c) {
            const int e = tid + c * 256;
            const int ly = e / C3_LX, lx = e - ly * C3_LX;
            const long q = e < C3_PL ? rule_index(a.g, a.P, a.plane, bx + lx - 1, by + ly - 1, z) : -1;
            const long qc = q < 0 ? 0 : q;
            const TC v = FIRST ? TC(a.b[qc]) * scale : TC(a.xk[qc]);
            r[c] = q >= 0 ? v : TC(0);
        }
    };
    auto put = [&](int z, const TC (&r)[NL]) {
        TC* buf = ring[z & 3];
#pragma unroll
        for (int c = 0; c < NL; ++c) {
            const int e = tid + c * 256;
            if (e < C3_PL) buf[e] = r[c];
        }
    };
    TC ra[NL], rb[NL];
    fetch(z0 - 1, ra);
    fetch(z0, rb);
    put(z0 - 1, ra);
    put(z0, rb);
    fetch(z0 + 1, ra);
    const TC alpha = TC(a.cf.alpha), b6 = TC(a.cf.beta * (1.0 / 6.0));
    const TC c1 = TC(a.c1), c2 = TC(a.c2);
    const int c0 = (ty + 1) * C3_LX + tx + 1;
    for (int z = z0; z < z1; ++z) {
        // the thread's own operands of plane z (index 0 for lanes outside)
        const size_t o = own ? (size_t)z * a.plane + (size_t)j * a.P + i : 0;
        const TC bv = TC(a.b[o]);
        // x_{k-1}: zero in the first pass, b / theta in the second
        const TC xp = (FIRST || OUT == C3_RESID) ? TC(0) : (a.xkm1 ? TC(a.xkm1[o]) : bv * TC(a.inv_theta));
        double fv = 0.0, gv = 0.0, cv = 0.0, av = 0.0;
        if (OUT == C3_FIELD) {
            fv = a.field[o];
            gv = a.ge ? a.ge[o] : 0.0;
            cv = a.ge ? a.cur[o] : 0.0;
            av = a.xadd ? (double)a.xadd[o] : 0.0;
        }
        // ring slot (z + 1) & 3 was last read in the iteration of plane z - 2
        put(z + 1, ra);
        if (z + 2 <= z1) fetch(z + 2, ra);
        __syncthreads();
        if (own) {
            const TC* pm = ring[(z - 1) & 3];
            const TC* pc = ring[z & 3];
            const TC* pp = ring[(z + 1) & 3];
            const TC xc = pc[c0];
            // faces: x, y in the plane and z across planes; edges: the four
            // in-plane diagonals and the x/y neighbours of the planes z +- 1
            const TC faces = pc[c0 - 1] + pc[c0 + 1] + pc[c0 - C3_LX] + pc[c0 + C3_LX] + pm[c0] + pp[c0];
            const TC edges = pc[c0 - C3_LX - 1] + pc[c0 - C3_LX + 1] + pc[c0 + C3_LX - 1] + pc[c0 + C3_LX + 1] +
                             pm[c0 - 1] + pm[c0 + 1] + pm[c0 - C3_LX] + pm[c0 + C3_LX] + pp[c0 - 1] + pp[c0 + 1] +
                             pp[c0 - C3_LX] + pp[c0 + C3_LX];
            const TC mx = fma(alpha, xc, -b6 * (TC(2) * faces + edges - TC(24) * xc));
            if (OUT == C3_RESID) {
                a.rout[o] = (float)(bv - mx);
            } else {
                const TC xn = xc + fma(c1, xc - xp, c2 * (bv - mx));
                if (OUT == C3_FIELD) {
                    const double phi = (double)xn + av;
                    const double de = a.cf.cfl * phi;
                    a.field[o] = fv + de;
                    if (a.ge) a.ge[o] = gv + fma(a.cf.ge_gain, de, -a.cf.ge_curl * cv);
                } else {
                    a.xout[o] = (TX)xn;
                }
            }
        }
    }
}

template <class TX, class TB, class TC, bool FIRST, int OUT>
__global__ __launch_bounds__(256) void k_cheb3t(Cheb3T<TX, TB> a)
{
    __shared__ TC ring[4][C3_PL];
    cheb3t_body<TX, TB, TC, FIRST, OUT>(a, make_uint3(blockIdx.x, blockIdx.y, blockIdx.z), ring);
}

static dim3 cheb3_grid(const UGrid& g)
{
    return dim3((unsigned)((g.hi[0] - g.lo[0] + C3_TX - 1) / C3_TX),
                (unsigned)((g.hi[1] - g.lo[1] + C3_TY - 1) / C3_TY),
                (unsigned)((g.hi[2] - g.lo[2] + C3_CZ - 1) / C3_CZ));
}

// Step sizes of the first-order Chebyshev form of K applications of M:
// x_1 = w_0 b, x_{k+1} = x_k + w_k (b - M x_k), w_j = 1 / mu_j at the K + 1
// roots mu_j of the Chebyshev polynomial on [alpha, alpha + 16 beta / 3].
// Its residual polynomial is that of the three-term recurrence with the
// same K applications, and no x_{k-1} is read.  Every factor 1 - lambda w_j
// stays below 3e-3 in size on the spectrum, so the order of the steps is
// free.
static void cheb_steps(const Coef& cf, int K, double* w)
{
    const double lmin = cf.alpha, lmax = cf.alpha + 16.0 / 3.0 * cf.beta;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    for (int j = 0; j <= K; ++j) w[j] = 1.0 / (theta - delta * cos((2 * j + 1) * M_PI / (2.0 * (K + 1))));
}

// One Chebyshev round of K passes on M x = b (the first-order form) with
// the iterates rotating through bufs[0..2].  Without a field the last pass stores x_{K+1} and the
// buffer holding it is returned; with a field the last pass applies
// field += cfl (x_{K+1} + xadd) and null is returned.
template <class TX, class TB, class TC>
static TX* cheb3_round(hipStream_t st, const Cheb3& c, const TB* b, TX* const* bufs, int K,
                       const Coef& cf, const TX* xadd, double* field, double* ge, const double* cur)
{
    const dim3 grid = cheb3_grid(c.g);
    TX* result = nullptr;
    double w[MAX_SWEEPS + 1];
    cheb_steps(cf, K, w);
    for (int k = 1; k <= K; ++k) {
        Cheb3T<TX, TB> a{};
        a.b = b;
        a.xk = bufs[k % 3];
        a.xkm1 = nullptr;                                 // not read: c1 = 0
        a.xout = bufs[(k + 1) % 3];
        a.xadd = xadd;
        a.field = field;
        a.ge = ge;
        a.cur = cur;
        a.g = c.g;
        a.P = c.P;
        a.plane = c.plane;
        a.inv_theta = w[0];                               // x_1 = w_0 b
        a.c1 = 0.0;
        a.c2 = w[k];
        a.cf = cf;
        const bool first = k == 1, last = k == K;
        if (last && field) {
            if (first) hipLaunchKernelGGL((k_cheb3t<TX, TB, TC, true, C3_FIELD>), grid, dim3(256), 0, st, a);
            else hipLaunchKernelGGL((k_cheb3t<TX, TB, TC, false, C3_FIELD>), grid, dim3(256), 0, st, a);
        } else {
            if (first) hipLaunchKernelGGL((k_cheb3t<TX, TB, TC, true, C3_STORE>), grid, dim3(256), 0, st, a);
            else hipLaunchKernelGGL((k_cheb3t<TX, TB, TC, false, C3_STORE>), grid, dim3(256), 0, st, a);
            if (last) result = bufs[(k + 1) % 3];
        }
    }
    return result;
}

hipError_t launch_solve3_mixed(hipStream_t st, const Cheb3& c, size_t arr, double* field, double* ge,
                               const double* cur, const Coef& cf, const ChebSchedule& cs)
{
    // FP32 views of the temporaries x, d0, d1: six arrays f[0..5]
    float* f[6];
    f[0] = reinterpret_cast<float*>(c.x);
    f[1] = f[0] + arr;
    f[2] = reinterpret_cast<float*>(c.d0);
    f[3] = f[2] + arr;
    f[4] = reinterpret_cast<float*>(c.d1);
    f[5] = f[4] + arr;
    const int s_round = (cs.sweeps - 1) / 2;
    float* r1[3] = {f[0], f[1], f[2]};
    float* x1 = cheb3_round<float, double, float>(st, c, c.r, r1, s_round, cf, nullptr, nullptr, nullptr,
                                                   nullptr);
    // res = b - M x1 in FP64 (x1 is exact in FP64), kept as FP32
    float* res = f[3];
    {
        Cheb3T<float, double> a{};
        a.b = c.r;
        a.xk = x1;
        a.rout = res;
        a.g = c.g;
        a.P = c.P;
        a.plane = c.plane;
        a.cf = cf;
        hipLaunchKernelGGL((k_cheb3t<float, double, double, false, C3_RESID>), cheb3_grid(c.g), dim3(256), 0, st,
                           a);
    }
    // second round: three buffers other than x1 and res
    float* r2[3];
    int n = 0;
    for (float* q : {f[0], f[1], f[2], f[4], f[5]})
        if (q != x1 && n < 3) r2[n++] = q;
    cheb3_round<float, float, float>(st, c, res, r2, s_round, cf, x1, field, ge, cur);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
// Segment of outputs per wave of k_march3: lines are cut so that a launch
// has at least about 8 waves per SIMD of the device.
static int march_segment(int n_out, long waves_per_seg)
{
    int seg = 256;
    while (seg > 32 && waves_per_seg * ((n_out + seg - 1) / seg) < 8192) seg /= 2;
    return seg;
}

template <int D>
static hipError_t launch_march_d(hipStream_t st, int mode, const Term3& t, double alpha, const PadeTaps& taps,
                                 const PadeLine& L)
{
    constexpr int T = 3 - D;
    const int nx = t.tg.hi[0] - t.tg.lo[0], nt = t.tg.hi[T] - t.tg.lo[T];
    const dim3 g0((nx + 63) / 64, (nt + 3) / 4, 1);
    const int seg = march_segment(L.n_out, (long)g0.x * g0.y * 4);
    const dim3 grid(g0.x, g0.y, (L.n_out + seg - 1) / seg);
    switch (mode) {
        case SRC_RAW: hipLaunchKernelGGL((k_march3<D, SRC_RAW>), grid, dim3(256), 0, st, t, alpha, taps, L, seg); break;
        case SRC_G: hipLaunchKernelGGL((k_march3<D, SRC_G>), grid, dim3(256), 0, st, t, alpha, taps, L, seg); break;
        case SRC_GE_STORED:
            hipLaunchKernelGGL((k_march3<D, SRC_GE_STORED>), grid, dim3(256), 0, st, t, alpha, taps, L, seg);
            break;
        default:
            hipLaunchKernelGGL((k_march3<D, SRC_GE_DISCRETE>), grid, dim3(256), 0, st, t, alpha, taps, L, seg);
            break;
    }
    return hipGetLastError();
}

template <int D>
static hipError_t launch_term_d(hipStream_t st, int mode, const Term3& t, double alpha, const PadeTaps& taps,
                                const PadeLine& L)
{
    constexpr int A = D == 0 ? 32 : 64;
    constexpr int NO = D == 0 ? 64 : 32;
    constexpr int W = D == 0 ? 1 : 0;
    constexpr int SX = 3 - D - W;
    dim3 grid((L.n_out + NO - 1) / NO, (t.tg.hi[W] - t.tg.lo[W] + A - 1) / A, t.tg.hi[SX] - t.tg.lo[SX]);
    switch (mode) {
        case SRC_RAW:
            hipLaunchKernelGGL((k_term3<D, SRC_RAW>), grid, dim3(256), 0, st, t, alpha, taps, L);
            break;
        case SRC_G: hipLaunchKernelGGL((k_term3<D, SRC_G>), grid, dim3(256), 0, st, t, alpha, taps, L); break;
        case SRC_GE_STORED:
            hipLaunchKernelGGL((k_term3<D, SRC_GE_STORED>), grid, dim3(256), 0, st, t, alpha, taps, L);
            break;
        default:
            hipLaunchKernelGGL((k_term3<D, SRC_GE_DISCRETE>), grid, dim3(256), 0, st, t, alpha, taps, L);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_condition3(hipStream_t st, int mode, const double* src, double* out, const Box& bx, int P,
                             size_t plane, double alpha)
{
    Term3 t{};
    t.src = src;
    t.out = out;
    t.sb = bx;
    t.P = P;
    t.plane = plane;
    const dim3 grid((bx.n[0] + 63) / 64, (bx.n[1] + 3) / 4, bx.n[2]);
    if (mode == SRC_G) hipLaunchKernelGGL((k_condition3<SRC_G>), grid, dim3(256), 0, st, t, alpha);
    else hipLaunchKernelGGL((k_condition3<SRC_GE_DISCRETE>), grid, dim3(256), 0, st, t, alpha);
    return hipGetLastError();
}

hipError_t launch_term3(hipStream_t st, int axis, int mode, const Term3& t, double alpha, const PadeTaps& taps,
                        const PadeLine& L)
{
    if (axis == 0) return launch_term_d<0>(st, mode, t, alpha, taps, L);
    if (axis == 1) return launch_march_d<1>(st, mode, t, alpha, taps, L);
    return launch_march_d<2>(st, mode, t, alpha, taps, L);
}

hipError_t launch_solve3(hipStream_t st, const Cheb3& c, double* field, double* ge, const double* cur,
                         const Coef& cf, const ChebSchedule& cs)
{
    // x_k rotates through three arrays: x, d0, d1 (b stays in r)
    double* bufs[3] = {c.x, c.d0, c.d1};
    cheb3_round<double, double, double>(st, c, c.r, bufs, cs.sweeps, cf, nullptr, field, ge, cur);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The recorded 3D step (Launch3): one problem's launches, in the order of
// Step 1 then Step 2 of Section 3.4 for the FP64 Chebyshev form, and the
// same launches over many problems.  A batched launch has one workgroup
// range per member ([first, first + gx gy gz)); the workgroup finds its
// member by a binary search over the range starts and runs the member's
// tile with the kernel body of the single-problem launch, so a member's
// results are those of the problem stepped alone.
// ---------------------------------------------------------------------------
struct TermB {
    Term3 t;
    PadeLine L;
    int seg;
    unsigned gx, gy;
    int first;
};
struct ChebB {
    Cheb3T<double, double> a;
    unsigned gx, gy;
    int first;
};

template <class B>
__device__ __forceinline__ uint3 member_block(const B* a, int count, int& m)
{
    const int b = (int)blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a[mid].first <= b) lo = mid;
        else hi = mid - 1;
    }
    m = lo;
    const unsigned local = (unsigned)(b - a[m].first), gx = a[m].gx, gy = a[m].gy;
    return make_uint3(local % gx, (local / gx) % gy, local / (gx * gy));
}

// The member's arguments are copied out of the table first: read through
// the table, every field would be reloaded after each store of the kernel
// (the stores could alias the table as far as the compiler knows).
template <int MODE>
__global__ __launch_bounds__(256) void k_condition3_b(const TermB* a, int count, double alpha)
{
    int m;
    const uint3 blk = member_block(a, count, m);
    const TermB arg = a[m];
    condition3_body<MODE>(arg.t, alpha, blk);
}

__global__ __launch_bounds__(256) void k_term3_b(const TermB* a, int count, double alpha, PadeTaps taps)
{
    __shared__ double sv[term3_lds<0>()];
    int m;
    const uint3 blk = member_block(a, count, m);
    const TermB arg = a[m];
    term3_body<0, SRC_RAW>(arg.t, alpha, taps, arg.L, blk, sv);
}

template <int D>
__global__ __launch_bounds__(256) void k_march3_b(const TermB* a, int count, double alpha, PadeTaps taps)
{
    int m;
    const uint3 blk = member_block(a, count, m);
    const TermB arg = a[m];
    march3_body<D, SRC_RAW>(arg.t, alpha, taps, arg.L, arg.seg, blk);
}

template <bool FIRST, int OUT>
__global__ __launch_bounds__(256) void k_cheb3t_b(const ChebB* a, int count)
{
    __shared__ double ring[4][C3_PL];
    int m;
    const uint3 blk = member_block(a, count, m);
    const ChebB arg = a[m];
    cheb3t_body<double, double, double, FIRST, OUT>(arg.a, blk, ring);
}

void plan_step3(const Plan3In& in, std::vector<Launch3>& out)
{
    out.clear();
    const double z = in.coef.z;
    double *b = in.tmp[0], *x = in.tmp[1], *d0 = in.tmp[2], *d1 = in.tmp[3], *cur = in.tmp[4];
    double* cond[3] = {in.tmp[5], in.tmp[6], in.tmp[7]};
    auto condition = [&](int first_src, int mode, int cls) {
        for (int j = 0; j < 3; ++j) {
            Launch3 r{};
            r.c.cf = in.coef;
            r.kind = L3_COND;
            r.mode = mode;
            r.cls = cls;
            r.group = 0;
            r.t.src = in.f[first_src + j];
            r.t.out = cond[j];
            r.t.sb = in.box[first_src + j];
            r.t.P = in.P;
            r.t.plane = in.plane;
            const Box& bx = in.box[first_src + j];
            r.gx = (unsigned)((bx.n[0] + 63) / 64);
            r.gy = (unsigned)((bx.n[1] + 3) / 4);
            r.gz = (unsigned)bx.n[2];
            out.push_back(r);
        }
    };
    auto term = [&](int axis, int src, const double* sp, double* o, double scale, int acc, int tgt, int line,
                    int cls, int group) {
        Launch3 r{};
        r.c.cf = in.coef;
        r.kind = axis == 0 ? L3_TERM : L3_MARCH;
        r.axis = axis;
        r.mode = SRC_RAW;
        r.line = line;
        r.cls = cls;
        r.group = group;
        r.t = Term3{sp, o, in.box[src], in.ug[tgt], in.P, in.plane, scale, acc};
        r.L = in.line[line];
        const UGrid& tg = r.t.tg;
        if (axis == 0) {
            r.gx = (unsigned)((r.L.n_out + 63) / 64);
            r.gy = (unsigned)((tg.hi[1] - tg.lo[1] + 31) / 32);
            r.gz = (unsigned)(tg.hi[2] - tg.lo[2]);
        } else {
            const int T = 3 - axis;
            const unsigned g0 = (unsigned)((tg.hi[0] - tg.lo[0] + 63) / 64), g1 = (unsigned)((tg.hi[T] - tg.lo[T] + 3) / 4);
            r.seg = march_segment(r.L.n_out, (long)g0 * g1 * 4);
            r.gx = g0;
            r.gy = g1;
            r.gz = (unsigned)((r.L.n_out + r.seg - 1) / r.seg);
        }
        out.push_back(r);
    };
    // the solve in the first-order form (cheb_steps)
    const int K = in.cheb.sweeps;
    double w[MAX_SWEEPS + 1];
    cheb_steps(in.coef, K, w);
    auto solve = [&](int comp, double* field, double* ge, const double* cr, int cls, int group) {
        double* bufs[3] = {x, d0, d1};
        for (int k = 1; k <= K; ++k) {
            Launch3 r{};
            r.kind = L3_CHEB;
            r.cls = cls;
            r.group = group;
            r.first = k == 1;
            const bool last = k == K;
            r.out = last ? C3_FIELD : C3_STORE;
            Cheb3T<double, double>& a = r.c;
            a.b = b;
            a.xk = bufs[k % 3];
            a.xkm1 = nullptr;                 // not read: c1 = 0
            a.xout = bufs[(k + 1) % 3];
            a.field = last ? field : nullptr;
            a.ge = last ? ge : nullptr;
            a.cur = last ? cr : nullptr;
            a.g = in.ug[comp];
            a.P = in.P;
            a.plane = in.plane;
            a.inv_theta = w[0];               // x_1 = w_0 b
            a.c1 = 0.0;
            a.c2 = w[k];
            a.cf = in.coef;
            const dim3 g = cheb3_grid(a.g);
            r.gx = g.x;
            r.gy = g.y;
            r.gz = g.z;
            out.push_back(r);
        }
    };
    // Step 1: conditioned H once, then per E component the line terms of
    // b (and of the raw curl with the carried Laplacian) and the solve
    condition(3, SRC_G, C4M_K_RHS_E);
    for (int c = 0; c < 3; ++c) {
        const int s1 = (c + 1) % 3, s2 = (c + 2) % 3;
        term(s1, 3 + s2, cond[s2], b, z, 0, c, 1, C4M_K_RHS_E, c);
        term(s2, 3 + s1, cond[s1], b, -z, 1, c, 1, C4M_K_RHS_E, c);
        if (in.tracked) {
            term(s1, 3 + s2, in.f[3 + s2], cur, 1.0, 0, c, 1, C4M_K_RHS_E, c);
            term(s2, 3 + s1, in.f[3 + s1], cur, -1.0, 1, c, 1, C4M_K_RHS_E, c);
        }
        solve(c, in.f[c], in.tracked ? in.ge[c] : nullptr, cur, C4M_K_SOLVE_E, c);
    }
    // Step 2: the stored G_E (or G(E) of the discrete Laplacian), per H component
    if (!in.tracked) condition(0, SRC_GE_DISCRETE, C4M_K_RHS_H);
    for (int c = 0; c < 3; ++c) {
        const int s1 = (c + 1) % 3, s2 = (c + 2) % 3;
        term(s1, s2, in.tracked ? in.ge[s2] : cond[s2], b, -1.0 / z, 0, 3 + c, 0, C4M_K_RHS_H, c);
        term(s2, s1, in.tracked ? in.ge[s1] : cond[s1], b, 1.0 / z, 1, 3 + c, 0, C4M_K_RHS_H, c);
        solve(3 + c, in.f[3 + c], nullptr, nullptr, C4M_K_SOLVE_H, c);
    }
}

hipError_t launch3_single(hipStream_t st, const Launch3& r, const PadeTaps* taps)
{
    const dim3 grid(r.gx, r.gy, r.gz), blk(256);
    switch (r.kind) {
        case L3_COND:
            if (r.mode == SRC_G) hipLaunchKernelGGL((k_condition3<SRC_G>), grid, blk, 0, st, r.t, r.c.cf.alpha);
            else hipLaunchKernelGGL((k_condition3<SRC_GE_DISCRETE>), grid, blk, 0, st, r.t, r.c.cf.alpha);
            break;
        case L3_TERM:
            hipLaunchKernelGGL((k_term3<0, SRC_RAW>), grid, blk, 0, st, r.t, r.c.cf.alpha, taps[r.line], r.L);
            break;
        case L3_MARCH:
            if (r.axis == 1)
                hipLaunchKernelGGL((k_march3<1, SRC_RAW>), grid, blk, 0, st, r.t, r.c.cf.alpha, taps[r.line], r.L, r.seg);
            else
                hipLaunchKernelGGL((k_march3<2, SRC_RAW>), grid, blk, 0, st, r.t, r.c.cf.alpha, taps[r.line], r.L, r.seg);
            break;
        default:
            if (r.first && r.out == C3_FIELD)
                hipLaunchKernelGGL((k_cheb3t<double, double, double, true, C3_FIELD>), grid, blk, 0, st, r.c);
            else if (r.first)
                hipLaunchKernelGGL((k_cheb3t<double, double, double, true, C3_STORE>), grid, blk, 0, st, r.c);
            else if (r.out == C3_FIELD)
                hipLaunchKernelGGL((k_cheb3t<double, double, double, false, C3_FIELD>), grid, blk, 0, st, r.c);
            else
                hipLaunchKernelGGL((k_cheb3t<double, double, double, false, C3_STORE>), grid, blk, 0, st, r.c);
            break;
    }
    return hipGetLastError();
}

size_t launch3_arg_bytes(const Launch3& r) { return r.kind == L3_CHEB ? sizeof(ChebB) : sizeof(TermB); }

void launch3_pack(const Launch3& r, int first_block, void* dst)
{
    if (r.kind == L3_CHEB) {
        ChebB c{};
        c.a = r.c;
        c.gx = r.gx;
        c.gy = r.gy;
        c.first = first_block;
        memcpy(dst, &c, sizeof(c));
    } else {
        TermB t{};
        t.t = r.t;
        t.L = r.L;
        t.seg = r.seg;
        t.gx = r.gx;
        t.gy = r.gy;
        t.first = first_block;
        memcpy(dst, &t, sizeof(t));
    }
}

hipError_t launch3_batched(hipStream_t st, const Launch3& proto, const void* dev_args, int count,
                           unsigned total_blocks, const PadeTaps* taps)
{
    const dim3 grid(total_blocks), blk(256);
    const TermB* tb = (const TermB*)dev_args;
    const ChebB* cb = (const ChebB*)dev_args;
    const double alpha = proto.c.cf.alpha;
    switch (proto.kind) {
        case L3_COND:
            if (proto.mode == SRC_G) hipLaunchKernelGGL((k_condition3_b<SRC_G>), grid, blk, 0, st, tb, count, alpha);
            else hipLaunchKernelGGL((k_condition3_b<SRC_GE_DISCRETE>), grid, blk, 0, st, tb, count, alpha);
            break;
        case L3_TERM:
            hipLaunchKernelGGL(k_term3_b, grid, blk, 0, st, tb, count, alpha, taps[proto.line]);
            break;
        case L3_MARCH:
            if (proto.axis == 1) hipLaunchKernelGGL((k_march3_b<1>), grid, blk, 0, st, tb, count, alpha, taps[proto.line]);
            else hipLaunchKernelGGL((k_march3_b<2>), grid, blk, 0, st, tb, count, alpha, taps[proto.line]);
            break;
        default:
            if (proto.first && proto.out == C3_FIELD)
                hipLaunchKernelGGL((k_cheb3t_b<true, C3_FIELD>), grid, blk, 0, st, cb, count);
            else if (proto.first)
                hipLaunchKernelGGL((k_cheb3t_b<true, C3_STORE>), grid, blk, 0, st, cb, count);
            else if (proto.out == C3_FIELD)
                hipLaunchKernelGGL((k_cheb3t_b<false, C3_FIELD>), grid, blk, 0, st, cb, count);
            else
                hipLaunchKernelGGL((k_cheb3t_b<false, C3_STORE>), grid, blk, 0, st, cb, count);
            break;
    }
    return hipGetLastError();
}

}  // namespace c4m
