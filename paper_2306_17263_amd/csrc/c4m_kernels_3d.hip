// c4m_kernels_3d.hip -- gfx950 kernels of the full 3D step (Ex..Hz).
//
// Step 1 (Section 3.4), per E component s (s1 = s+1, s2 = s+2 mod 3):
//   b   = Z (delta_{s1} G(H_{s2}) - delta_{s2} G(H_{s1}))      k_term3 twice
//   c   = delta_{s1} H_{s2} - delta_{s2} H_{s1}                 (carried l) k_term3 twice
//   Phi = M^{-1} b (19-point M), E_s += r Phi, G_E += ...       k_cheb3t
// Step 2, per H component s:
//   b   = -(1/Z) (delta_{s1} G_{E,s2} - delta_{s2} G_{E,s1}),   H_s += r M^{-1} b.
//
// k_term3: one Pade line derivative along axis D, accumulated into the
// target's right-hand side.  A tile holds A lines of the target (32 rows
// along y for D = x, 64 columns along x otherwise) with 32 or 64 outputs
// each; the conditioned source values of the tile's line windows are staged
// in LDS (coalesced loads), then every thread runs the truncated Pade FIR
// over a register window of 8 consecutive outputs.
//
// Chebyshev (FP64): three-term form, one z-marching launch per application
// of M with the planes of the iterate staged in LDS (k_cheb3t).  The
// FP32-refined form runs its two FP32 rounds as per-sweep kernels on FP32
// views of the temporaries (k_cheb3f_*).
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

// Source value at stored index q (q[D] may run outside the line: zero).
// SRC_G: alpha u + (sum of second differences)/12 with even ghosts along
// half axes (node axes are interior here); SRC_GE_DISCRETE: the same on E,
// zero on E's node walls.
template <int MODE>
__device__ __forceinline__ double src_value(const Term3& t, int i, int j, int k, double alpha)
{
    const Box& b = t.sb;
    if (i < 0 || j < 0 || k < 0 || i >= b.n[0] || j >= b.n[1] || k >= b.n[2]) return 0.0;
    const double* p = t.src + k * t.plane + (size_t)j * t.P + i;
    if (MODE == SRC_RAW || MODE == SRC_GE_STORED) return p[0];
    const int q[3] = {i, j, k};
    const size_t st[3] = {1, (size_t)t.P, t.plane};
    if (MODE == SRC_GE_DISCRETE) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
            if (!b.half[d] && (q[d] == 0 || q[d] == b.n[d] - 1)) return 0.0;
    }
    const double u0 = p[0];
    double lap = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double um = q[d] == 0 ? u0 : p[-(long)st[d]];          // even ghost (half axis)
        const double up = q[d] == b.n[d] - 1 ? u0 : p[st[d]];
        lap += um + up - 2.0 * u0;
    }
    return fma(alpha, u0, lap * (1.0 / 12.0));
}

constexpr int T3_SEG = 8;

template <int D, int MODE>
__global__ __launch_bounds__(256) void k_term3(Term3 t, double alpha, PadeTaps taps, PadeLine L)
{
    // tile geometry: A lines x NO outputs per line
    constexpr int A = D == 0 ? 32 : 64;
    constexpr int NO = D == 0 ? 64 : 32;
    constexpr int BW = NO + PADE_TAPS - 1;       // staged window per line
    constexpr int BS = (BW % 2) ? BW : BW + 1;   // odd stride
    __shared__ double sv[A * BS];
    // axes: D = line axis, W = across lines in the tile, Sx = slab (blockIdx.z)
    constexpr int W = D == 0 ? 1 : 0;
    constexpr int SX = 3 - D - W;
    const int m0 = blockIdx.x * NO;                       // first output along D
    const int w0 = t.tg.lo[W] + blockIdx.y * A;           // first line along W
    const int s = t.tg.lo[SX] + blockIdx.z;               // slab index
    const int tid = threadIdx.x;
    const int n_in = L.n_in;
    for (int e = tid; e < A * BW; e += 256) {
        int a, q;
        if (D == 0) { a = e / BW; q = e - a * BW; }       // consecutive threads along the line (x)
        else { q = e / A; a = e - q * A; }                // consecutive threads across lines (x)
        const int wi = w0 + a;
        const int g = m0 - PADE_R + q;
        double v = 0.0;
        if (wi < t.tg.hi[W] && g >= 0 && g < n_in) {
            int idx[3];
            idx[D] = g;
            idx[W] = wi;
            idx[SX] = s;
            v = src_value<MODE>(t, idx[0], idx[1], idx[2], alpha);
        }
        sv[a * BS + q] = v;
    }
    __syncthreads();
    // thread -> (line a, segment): lanes of a half-wave take consecutive lines
    const int a = tid % A;
    const int seg = tid / A;
    const int mb = m0 + seg * T3_SEG;
    const double* w = sv + a * BS + seg * T3_SEG;
    double out[T3_SEG];
    const bool fast = !L.all && mb >= L.b && mb + T3_SEG - 1 < L.n_out - L.b;
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
        double* o = t.out + idx[2] * t.plane + (size_t)idx[1] * t.P + idx[0];
        const double v = t.scale * out[k];
        *o = t.accumulate ? *o + v : v;
    }
}

// ---------------------------------------------------------------------------
// Chebyshev sweeps on one component grid.
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool cell3(const UGrid& g, int& i, int& j, int& k)
{
    const int nx = g.hi[0] - g.lo[0], ny = g.hi[1] - g.lo[1], nz = g.hi[2] - g.lo[2];
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)nx * ny * nz) return false;
    i = g.lo[0] + (int)(e % nx);
    const long rest = e / nx;
    j = g.lo[1] + (int)(rest % ny);
    k = g.lo[2] + (int)(rest / ny);
    return true;
}

// ---------------------------------------------------------------------------
// FP64 solve: Chebyshev in three-term form on the same schedule,
//   x_1 = b / theta,  x_{k+1} = x_k + c1_{k-1} (x_k - x_{k-1}) + c2_{k-1} (b - M x_k),
// k = 1..K, Phi = x_{K+1} (K applications of M).  Each application is one
// z-marching pass over the grid: a workgroup owns a 64 x 4 column tile and
// a chunk of planes, and keeps the three planes z-1, z, z+1 of x_k (with a
// one-point ring, boundary rules applied when loading) in a 4-deep LDS ring.
// The first pass reads only b; the last writes the field update.
// ---------------------------------------------------------------------------
constexpr int C3_TX = 64, C3_TY = 4, C3_CZ = 16;
constexpr int C3_LX = C3_TX + 2, C3_LY = C3_TY + 2, C3_PL = C3_LX * C3_LY;

struct Cheb3T {
    const double* b;
    const double* xk;       // x_k (unused in the first pass: x_1 = b / theta)
    const double* xkm1;     // x_{k-1} (unused in the first pass: x_0 = 0)
    double* xout;           // x_{k+1} (unused in the last pass)
    double* field;          // last pass: field += cfl Phi
    double* ge;             // last pass, carried Laplacian: G_E update (or null)
    const double* cur;      // raw curl for the G_E update
    UGrid g;
    int P;
    size_t plane;
    double inv_theta, c1, c2;
    Coef cf;
};

// Index of grid point (i, j, k) after the boundary rules of the unknowns:
// Dirichlet outside the range -> -1 (zero), Neumann -> mirrored onto the
// edge unknown.
__device__ __forceinline__ long rule_index(const Cheb3T& a, int i, int j, int k)
{
    int q[3] = {i, j, k};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (q[d] < a.g.lo[d]) {
            if (!a.g.neumann[d]) return -1;
            q[d] = a.g.lo[d];
        } else if (q[d] >= a.g.hi[d]) {
            if (!a.g.neumann[d]) return -1;
            q[d] = a.g.hi[d] - 1;
        }
    }
    return (long)q[2] * (long)a.plane + (long)q[1] * a.P + q[0];
}

template <bool FIRST, bool LAST>
__global__ __launch_bounds__(256) void k_cheb3t(Cheb3T a)
{
    __shared__ double ring[4][C3_PL];
    const int tid = threadIdx.x;
    const int tx = tid % C3_TX, ty = tid / C3_TX;
    const int bx = a.g.lo[0] + blockIdx.x * C3_TX, by = a.g.lo[1] + blockIdx.y * C3_TY;
    const int i = bx + tx, j = by + ty;
    const int z0 = a.g.lo[2] + blockIdx.z * C3_CZ;
    const int z1 = min(z0 + C3_CZ, a.g.hi[2]);
    const bool own = i < a.g.hi[0] && j < a.g.hi[1];
    const double* src = FIRST ? a.b : a.xk;
    const double scale = FIRST ? a.inv_theta : 1.0;
    auto load = [&](int z) {
        double* buf = ring[z & 3];
        for (int e = tid; e < C3_PL; e += 256) {
            const int ly = e / C3_LX, lx = e - ly * C3_LX;
            const long q = rule_index(a, bx + lx - 1, by + ly - 1, z);
            buf[e] = q < 0 ? 0.0 : scale * src[q];
        }
    };
    load(z0 - 1);
    load(z0);
    const double b6 = a.cf.beta * (1.0 / 6.0);
    const int c0 = (ty + 1) * C3_LX + tx + 1;
    for (int z = z0; z < z1; ++z) {
        load(z + 1);
        __syncthreads();
        if (own) {
            const double* pm = ring[(z - 1) & 3];
            const double* pc = ring[z & 3];
            const double* pp = ring[(z + 1) & 3];
            const double xc = pc[c0];
            // faces: x, y in the plane and z across planes; edges: the four
            // in-plane diagonals and the x/y neighbours of the planes z +- 1
            const double faces = pc[c0 - 1] + pc[c0 + 1] + pc[c0 - C3_LX] + pc[c0 + C3_LX] + pm[c0] + pp[c0];
            const double edges = pc[c0 - C3_LX - 1] + pc[c0 - C3_LX + 1] + pc[c0 + C3_LX - 1] +
                                 pc[c0 + C3_LX + 1] + pm[c0 - 1] + pm[c0 + 1] + pm[c0 - C3_LX] +
                                 pm[c0 + C3_LX] + pp[c0 - 1] + pp[c0 + 1] + pp[c0 - C3_LX] + pp[c0 + C3_LX];
            const double mx = fma(a.cf.alpha, xc, -b6 * (2.0 * faces + edges - 24.0 * xc));
            const size_t o = (size_t)z * a.plane + (size_t)j * a.P + i;
            const double bv = a.b[o];
            const double xp = FIRST ? 0.0 : a.xkm1[o];
            const double xn = xc + fma(a.c1, xc - xp, a.c2 * (bv - mx));
            if (LAST) {
                const double de = a.cf.cfl * xn;
                a.field[o] += de;
                if (a.ge) a.ge[o] += fma(a.cf.ge_gain, de, -a.cf.ge_curl * a.cur[o]);
            } else {
                a.xout[o] = xn;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Mixed precision: two FP32 rounds x1 = C(b), x2 = C(b - M x1) around one
// FP64 residual; the round arrays are FP32 views of the FP64 temporaries.
// ---------------------------------------------------------------------------
struct Cheb3f {
    float* r;
    float* x;
    float* d0;
    float* d1;
    UGrid g;
    int P;
    size_t plane;
};

__device__ __forceinline__ float dvalf(const Cheb3f& c, const float* d, int i, int j, int k)
{
    int q[3] = {i, j, k};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (q[a] < c.g.lo[a]) {
            if (!c.g.neumann[a]) return 0.f;
            q[a] = c.g.lo[a];
        } else if (q[a] >= c.g.hi[a]) {
            if (!c.g.neumann[a]) return 0.f;
            q[a] = c.g.hi[a] - 1;
        }
    }
    return d[q[2] * c.plane + (size_t)q[1] * c.P + q[0]];
}

template <class T, class V>
__device__ __forceinline__ T l9_3d(const V& c, const T* d, int i, int j, int k, T (*val)(const V&, const T*, int, int, int))
{
    T faces = 0, edges = 0;
    faces += val(c, d, i - 1, j, k) + val(c, d, i + 1, j, k);
    faces += val(c, d, i, j - 1, k) + val(c, d, i, j + 1, k);
    faces += val(c, d, i, j, k - 1) + val(c, d, i, j, k + 1);
    for (int a = -1; a <= 1; a += 2)
        for (int b = -1; b <= 1; b += 2) {
            edges += val(c, d, i + a, j + b, k);
            edges += val(c, d, i, j + a, k + b);
            edges += val(c, d, i + a, j, k + b);
        }
    return (T(2) * faces + edges - T(24) * d[k * c.plane + (size_t)j * c.P + i]) * T(1.0 / 6.0);
}

// r32 = (float) src, d = r32 / theta, x = 0
__global__ void k_cheb3f_init2(Cheb3f c, const float* __restrict__ src, float inv_theta)
{
    int i, j, k;
    if (!cell3(c.g, i, j, k)) return;
    const size_t o = k * c.plane + (size_t)j * c.P + i;
    const float r0 = src[o];
    c.r[o] = r0;
    c.d0[o] = r0 * inv_theta;
    c.x[o] = 0.f;
}

__global__ void k_cheb3f_init(Cheb3f c, const double* __restrict__ src, float inv_theta)
{
    int i, j, k;
    if (!cell3(c.g, i, j, k)) return;
    const size_t o = k * c.plane + (size_t)j * c.P + i;
    const float r0 = (float)src[o];
    c.r[o] = r0;
    c.d0[o] = r0 * inv_theta;
    c.x[o] = 0.f;
}

__global__ void k_cheb3f_sweep(Cheb3f c, const float* __restrict__ din, float* __restrict__ dout, float alpha,
                               float beta, float c1, float c2, int last)
{
    int i, j, k;
    if (!cell3(c.g, i, j, k)) return;
    const size_t o = k * c.plane + (size_t)j * c.P + i;
    const float dc = din[o];
    const float ad = fmaf(alpha, dc, -beta * l9_3d<float, Cheb3f>(c, din, i, j, k, dvalf));
    const float x = c.x[o] + dc;
    const float rn = c.r[o] - ad;
    c.r[o] = rn;
    const float dn = fmaf(c1, dc, c2 * rn);
    dout[o] = dn;
    c.x[o] = last ? x + dn : x;          // the last sweep folds in x_{K+1} = x_K + d_K
}

__device__ __forceinline__ double dval1(const Cheb3f& c, const float* d, int i, int j, int k)
{
    return (double)dvalf(c, d, i, j, k);
}

// res = b - M x1 in FP64 (x1 is exactly representable), stored as FP32
__global__ void k_cheb3f_resid(Cheb3f c, const double* __restrict__ b, const float* __restrict__ x1,
                               float* __restrict__ res, double alpha, double beta)
{
    int i, j, k;
    if (!cell3(c.g, i, j, k)) return;
    const size_t o = k * c.plane + (size_t)j * c.P + i;
    double faces = 0, edges = 0;
    faces += dval1(c, x1, i - 1, j, k) + dval1(c, x1, i + 1, j, k);
    faces += dval1(c, x1, i, j - 1, k) + dval1(c, x1, i, j + 1, k);
    faces += dval1(c, x1, i, j, k - 1) + dval1(c, x1, i, j, k + 1);
    for (int a = -1; a <= 1; a += 2)
        for (int bb = -1; bb <= 1; bb += 2) {
            edges += dval1(c, x1, i + a, j + bb, k);
            edges += dval1(c, x1, i, j + a, k + bb);
            edges += dval1(c, x1, i + a, j, k + bb);
        }
    const double xc = (double)x1[o];
    const double l9 = (2.0 * faces + edges - 24.0 * xc) * (1.0 / 6.0);
    res[o] = (float)(b[o] - fma(alpha, xc, -beta * l9));
}

__global__ void k_cheb3f_final(Cheb3f c, const float* __restrict__ x1, const float* __restrict__ x2, double* field,
                               double* ge, const double* cur, Coef cf)
{
    int i, j, k;
    if (!cell3(c.g, i, j, k)) return;
    const size_t o = k * c.plane + (size_t)j * c.P + i;
    const double de = cf.cfl * ((double)x1[o] + (double)x2[o]);
    field[o] += de;
    if (ge) ge[o] += fma(cf.ge_gain, de, -cf.ge_curl * cur[o]);
}

hipError_t launch_solve3_mixed(hipStream_t st, const Cheb3& c, size_t arr, double* field, double* ge,
                               const double* cur, const Coef& cf, const ChebSchedule& cs)
{
    const long cells = (long)(c.g.hi[0] - c.g.lo[0]) * (c.g.hi[1] - c.g.lo[1]) * (c.g.hi[2] - c.g.lo[2]);
    const dim3 grid((unsigned)((cells + 255) / 256));
    // FP32 views: x1 | x2 in the x array, d0 | d1 in d0, the round residual in d1
    float* x1 = reinterpret_cast<float*>(c.x);
    float* x2 = x1 + arr;
    float* d0 = reinterpret_cast<float*>(c.d0);
    float* d1 = d0 + arr;
    float* rr = reinterpret_cast<float*>(c.d1);
    float* res = rr + arr;
    const int s_round = (cs.sweeps - 1) / 2;
    for (int round = 0; round < 2; ++round) {
        Cheb3f f{rr, round == 0 ? x1 : x2, d0, d1, c.g, c.P, c.plane};
        if (round == 0)
            hipLaunchKernelGGL(k_cheb3f_init, grid, dim3(256), 0, st, f, (const double*)c.r, cs.inv_thetaf);
        else {
            hipLaunchKernelGGL(k_cheb3f_resid, grid, dim3(256), 0, st, f, (const double*)c.r, x1, res, cf.alpha,
                               cf.beta);
            // round 2 starts from the residual (kept in FP32)
            hipLaunchKernelGGL(k_cheb3f_init2, grid, dim3(256), 0, st, f, res, cs.inv_thetaf);
        }
        float* din = d0;
        float* dout = d1;
        for (int k = 0; k < s_round; ++k) {
            hipLaunchKernelGGL(k_cheb3f_sweep, grid, dim3(256), 0, st, f, din, dout, (float)cf.alpha, (float)cf.beta,
                               cs.c1f[k], cs.c2f[k], k == s_round - 1 ? 1 : 0);
            float* tmp = din;
            din = dout;
            dout = tmp;
        }
    }
    hipLaunchKernelGGL(k_cheb3f_final, grid, dim3(256), 0, st, Cheb3f{rr, x1, d0, d1, c.g, c.P, c.plane}, x1, x2,
                       field, ge, cur, cf);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
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
        case SRC_RAW: hipLaunchKernelGGL((k_term3<D, SRC_RAW>), grid, dim3(256), 0, st, t, alpha, taps, L); break;
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

hipError_t launch_term3(hipStream_t st, int axis, int mode, const Term3& t, double alpha, const PadeTaps& taps,
                        const PadeLine& L)
{
    if (axis == 0) return launch_term_d<0>(st, mode, t, alpha, taps, L);
    if (axis == 1) return launch_term_d<1>(st, mode, t, alpha, taps, L);
    return launch_term_d<2>(st, mode, t, alpha, taps, L);
}

hipError_t launch_solve3(hipStream_t st, const Cheb3& c, double* field, double* ge, const double* cur,
                         const Coef& cf, const ChebSchedule& cs)
{
    const dim3 grid((unsigned)((c.g.hi[0] - c.g.lo[0] + C3_TX - 1) / C3_TX),
                    (unsigned)((c.g.hi[1] - c.g.lo[1] + C3_TY - 1) / C3_TY),
                    (unsigned)((c.g.hi[2] - c.g.lo[2] + C3_CZ - 1) / C3_CZ));
    // x_k rotates through three arrays: x, d0, d1 (b stays in r)
    double* bufs[3] = {c.x, c.d0, c.d1};
    const int K = cs.sweeps;
    for (int k = 1; k <= K; ++k) {
        Cheb3T a{};
        a.b = c.r;
        a.xk = bufs[k % 3];
        a.xkm1 = bufs[(k - 1) % 3];
        a.xout = bufs[(k + 1) % 3];
        a.field = field;
        a.ge = ge;
        a.cur = cur;
        a.g = c.g;
        a.P = c.P;
        a.plane = c.plane;
        a.inv_theta = cs.inv_theta;
        a.c1 = cs.c1[k - 1];
        a.c2 = cs.c2[k - 1];
        a.cf = cf;
        const bool first = k == 1, last = k == K;
        if (first && last) hipLaunchKernelGGL((k_cheb3t<true, true>), grid, dim3(256), 0, st, a);
        else if (first) hipLaunchKernelGGL((k_cheb3t<true, false>), grid, dim3(256), 0, st, a);
        else if (last) hipLaunchKernelGGL((k_cheb3t<false, true>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_cheb3t<false, false>), grid, dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace c4m
