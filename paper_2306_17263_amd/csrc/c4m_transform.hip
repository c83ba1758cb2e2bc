// c4m_transform.hip -- direct solve of M = alpha I - beta L9 by sine and
// cosine transforms (Appendix A.2, Def. def:operatorsP).
//
// Along a node axis of a component (Dirichlet: unknowns 1..N-1) the second
// difference is diagonal in the sine modes sin(pi k j / N), k = 1..N-1
// (DST-I); along a half-point axis (Neumann, even ghost: unknowns 0..N-1)
// in the cosine modes cos(pi k (j + 1/2) / N), k = 0..N-1 (DCT-II); both
// with eigenvalue -sigma_k, sigma_k = 4 sin^2(pi k / 2N).  L9 is the sum of
// the second differences plus one sixth of their pairwise products, so M is
// diagonal in the product basis:
//   lambda = alpha + beta (sum sigma - (sum over pairs sigma sigma) / 6).
// The solve applies the orthonormal transform matrix of each axis (a dense
// contraction over a whole line), divides by lambda and transforms back:
// 2D four matrix products, 3D six, each one launch of k_gemm_f64 on the
// FP64 matrix cores.  The division by lambda rides in the epilogue of the
// last forward product, the field (and G_E) update in that of the last
// inverse one, so b is read once and the field read-modify-written once.
//
// k_gemm_f64: C = A B (row-major, leading dimensions, a batch index with
// strides).  A 256-thread workgroup owns a 64 x BN tile of C (BN = 64, or
// 128 for the long products of 2D); each of its four waves a 32 x BN/2
// quarter as 2 x BN/32 tiles of v_mfma_f64_16x16x4f64, whose operands are
// laid out as: lane l holds A[l % 16][l / 16] of a 16 x 4 block and
// B[l / 16][l % 16] of a 4 x 16 block, and value i of the accumulator is
// C[l / 16 + 4 i][l % 16].  K advances in steps of 16 through LDS (A as
// [64][17], B as [16][BN + 1] to spread the banks); the next step's global
// loads are in flight while the matrix cores work on the current one.
#include "c4m_internal.h"

namespace c4m {

typedef double v4d __attribute__((ext_vector_type(4)));

enum { EPI_STORE = 0, EPI_LAMBDA = 1, EPI_FIELD = 2 };

struct GemmArgs {
    const double* a;
    const double* b;
    double* c;
    long lda, ldb, ldc;
    long sa, sb, sc;          // batch strides
    int m, n, k;
    // EPI_LAMBDA: c = (A B) / lambda at (kz, ky, kx) of the unknown grid;
    // three_d: kz = row, (ky, kx) = (col / nx, col % nx); else (ky, kx) = (row, col)
    const double* sig[3];     // sigma of the x, y, z transform axes (null: inactive)
    int nx, three_d;
    double alpha, beta;
    // EPI_FIELD: field[o] += cfl v, o = batch * plane + row * P + col + off
    double* field;
    double* ge;
    const double* cur;
    long P, plane, off;
    double cfl, ge_gain, ge_curl;
};

constexpr int G_BM = 64, G_BK = 16;
constexpr int G_AS = G_BK + 1;

template <int EPI, int G_BN>
__global__ __launch_bounds__(256) void k_gemm_f64(GemmArgs g)
{
    constexpr int G_WN = G_BN / 32;      // 16-column MFMA tiles per wave
    constexpr int G_BS = G_BN + 1;
    __shared__ double As[G_BM * G_AS];
    __shared__ double Bs[G_BK * G_BS];
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const int m0 = blockIdx.y * G_BM, n0 = blockIdx.x * G_BN, bz = blockIdx.z;
    const double* A = g.a + bz * g.sa;
    const double* B = g.b + bz * g.sb;
    const int wm = (wave / 2) * 32, wn = (wave % 2) * (G_BN / 2);   // the wave's quarter
    v4d acc[2][G_WN];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < G_WN; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    // stage A[m0 .. +64][k0 .. +16] and B[k0 .. +16][n0 .. +64] (zero
    // outside) into registers; the next tile's loads are issued before the
    // current tile's products, so they are in flight while the matrix cores
    // work
    constexpr int NB = G_BK * G_BN / 256;
    double va[4], vb[NB];
    auto load = [&](int k0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int e = tid + c * 256;
            const int ar = e / G_BK, ac = e % G_BK;
            const int gr = m0 + ar, gc = k0 + ac;
            va[c] = (gr < g.m && gc < g.k) ? A[gr * g.lda + gc] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const int e = tid + c * 256;
            const int br = e / G_BN, bc = e % G_BN;
            const int hr = k0 + br, hc = n0 + bc;
            vb[c] = (hr < g.k && hc < g.n) ? B[hr * g.ldb + hc] : 0.0;
        }
    };
    load(0);
    for (int k0 = 0; k0 < g.k; k0 += G_BK) {
        __syncthreads();   // the previous tile's products have read the LDS
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int e = tid + c * 256;
            As[(e / G_BK) * G_AS + e % G_BK] = va[c];
        }
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const int e = tid + c * 256;
            Bs[(e / G_BN) * G_BS + e % G_BN] = vb[c];
        }
        __syncthreads();
        if (k0 + G_BK < g.k) load(k0 + G_BK);
#pragma unroll
        for (int kk = 0; kk < G_BK; kk += 4) {
            double fa[2], fb[G_WN];
#pragma unroll
            for (int i = 0; i < 2; ++i) fa[i] = As[(wm + i * 16 + lane % 16) * G_AS + kk + lane / 16];
#pragma unroll
            for (int j = 0; j < G_WN; ++j) fb[j] = Bs[(kk + lane / 16) * G_BS + wn + j * 16 + lane % 16];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < G_WN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fb[j], acc[i][j], 0, 0, 0);
        }
    }
    // epilogue
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < G_WN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm + i * 16 + lane / 16 + 4 * v;
                const int col = n0 + wn + j * 16 + lane % 16;
                if (row >= g.m || col >= g.n) continue;
                double val = acc[i][j][v];
                if (EPI == EPI_LAMBDA) {
                    int kz, ky, kx;
                    if (g.three_d) {
                        kz = row;
                        ky = col / g.nx;
                        kx = col - ky * g.nx;
                    } else {
                        kz = 0;
                        ky = row;
                        kx = col;
                    }
                    const double sx = g.sig[0] ? g.sig[0][kx] : 0.0;
                    const double sy = g.sig[1] ? g.sig[1][ky] : 0.0;
                    const double sz = g.sig[2] ? g.sig[2][kz] : 0.0;
                    const double lam =
                        g.alpha + g.beta * ((sx + sy + sz) - (sx * sy + sx * sz + sy * sz) * (1.0 / 6.0));
                    g.c[bz * g.sc + row * g.ldc + col] = val / lam;
                } else if (EPI == EPI_FIELD) {
                    const long o = bz * g.plane + row * g.P + col + g.off;
                    const double de = g.cfl * val;
                    g.field[o] += de;
                    if (g.ge) g.ge[o] += fma(g.ge_gain, de, -g.ge_curl * g.cur[o]);
                } else {
                    g.c[bz * g.sc + row * g.ldc + col] = val;
                }
            }
}

template <int BN>
static void gemm_launch(hipStream_t st, int epi, const GemmArgs& g, int batch)
{
    const dim3 grid((g.n + BN - 1) / BN, (g.m + G_BM - 1) / G_BM, batch);
    if (epi == EPI_LAMBDA) hipLaunchKernelGGL((k_gemm_f64<EPI_LAMBDA, BN>), grid, dim3(256), 0, st, g);
    else if (epi == EPI_FIELD) hipLaunchKernelGGL((k_gemm_f64<EPI_FIELD, BN>), grid, dim3(256), 0, st, g);
    else hipLaunchKernelGGL((k_gemm_f64<EPI_STORE, BN>), grid, dim3(256), 0, st, g);
}

// 64 x 128 tiles for long products (the 2D transforms, K = N), 64 x 64 for
// the short ones of 3D (measured: 2D 47.8 -> 50.0, 3D 40.5 -> 37.8 TFLOP/s
// with 64 x 128 everywhere)
static hipError_t gemm(hipStream_t st, int epi, const GemmArgs& g, int batch)
{
    if (g.k >= 1024) gemm_launch<128>(st, epi, g, batch);
    else gemm_launch<64>(st, epi, g, batch);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tables: for N, the orthonormal DST-I matrix S (N-1 x N-1, symmetric), the
// DCT-II matrix C (N x N) and its transpose, and sigma of both kinds.
// ---------------------------------------------------------------------------
size_t transform_table_doubles(int N)
{
    const size_t nd = (size_t)(N - 1), nn = (size_t)N;
    return nd * nd + 2 * nn * nn + nd + nn;
}

void build_transform_tables(int N, double* h, TransformTables* t, double* dev)
{
    const size_t nd = (size_t)(N - 1), nn = (size_t)N;
    double* S = h;
    double* C = S + nd * nd;
    double* Ct = C + nn * nn;
    double* sd = Ct + nn * nn;
    double* sn = sd + nd;
    const double pi = 3.14159265358979323846;
    for (size_t k = 0; k < nd; ++k)
        for (size_t j = 0; j < nd; ++j) {
            // sin(pi (k+1)(j+1) / N) with the product reduced mod 2N (exact in integers)
            const long q = (long)((k + 1) * (j + 1) % (2 * nn));
            S[k * nd + j] = sqrt(2.0 / N) * sin(pi * (double)q / N);
        }
    for (size_t k = 0; k < nn; ++k)
        for (size_t j = 0; j < nn; ++j) {
            // cos(pi k (2 j + 1) / 2N), argument reduced mod 4N
            const long q = (long)(k * (2 * j + 1) % (4 * nn));
            const double v = (k == 0 ? sqrt(1.0 / N) : sqrt(2.0 / N)) * cos(pi * (double)q / (2.0 * N));
            C[k * nn + j] = v;
            Ct[j * nn + k] = v;
        }
    for (size_t k = 0; k < nd; ++k) {
        const double s = sin(pi * (double)(k + 1) / (2.0 * N));
        sd[k] = 4.0 * s * s;
    }
    for (size_t k = 0; k < nn; ++k) {
        const double s = sin(pi * (double)k / (2.0 * N));
        sn[k] = 4.0 * s * s;
    }
    t->S = dev;
    t->C = dev + (C - h);
    t->Ct = dev + (Ct - h);
    t->sig_d = dev + (sd - h);
    t->sig_n = dev + (sn - h);
}

// x = M^{-1} b on the unknowns g of one component (b in the padded layout,
// read only), then field += cfl x (and the G_E update when ge is given);
// w1, w2: dense work arrays of the unknown count.
hipError_t launch_transform_solve(hipStream_t st, int dim, const TransformTables& t, const UGrid& g, int P,
                                  size_t plane, const double* b, double* w1, double* w2, double* field, double* ge,
                                  const double* cur, const Coef& cf)
{
    int n[3];
    const double* T[3];     // forward matrix per axis
    const double* Ti[3];    // inverse (transpose)
    const double* sg[3];
    for (int d = 0; d < 3; ++d) {
        n[d] = g.hi[d] - g.lo[d];
        if (d >= dim) {
            T[d] = Ti[d] = sg[d] = nullptr;
            continue;
        }
        if (g.neumann[d]) {
            T[d] = t.C;
            Ti[d] = t.Ct;
            sg[d] = t.sig_n;
        } else {
            T[d] = t.S;
            Ti[d] = t.S;
            sg[d] = t.sig_d;
        }
    }
    const int nx = n[0], ny = n[1], nz = dim == 3 ? n[2] : 1;
    const long off = (long)g.lo[2] * (long)plane + (long)g.lo[1] * P + g.lo[0];
    const long pl = (long)ny * nx;
    hipError_t e;
    // forward along x: W1[z][j][k] = sum_i b[z][j][i] Tx[k][i]  (B operand Tx^T)
    {
        GemmArgs a{};
        a.a = b + off;
        a.lda = P;
        a.sa = (long)plane;
        a.b = Ti[0];
        a.ldb = nx;
        a.c = w1;
        a.ldc = nx;
        a.sc = pl;
        a.m = ny;
        a.n = nx;
        a.k = nx;
        e = gemm(st, EPI_STORE, a, nz);
        if (e != hipSuccess) return e;
    }
    // forward along y: W2[z] = Ty W1[z]  (3D; in 2D this product divides by lambda)
    {
        GemmArgs a{};
        a.a = T[1];
        a.lda = ny;
        a.b = w1;
        a.ldb = nx;
        a.sb = pl;
        a.c = w2;
        a.ldc = nx;
        a.sc = pl;
        a.m = ny;
        a.n = nx;
        a.k = ny;
        a.sig[0] = sg[0];
        a.sig[1] = sg[1];
        a.nx = nx;
        a.alpha = cf.alpha;
        a.beta = cf.beta;
        e = gemm(st, dim == 2 ? EPI_LAMBDA : EPI_STORE, a, nz);
        if (e != hipSuccess) return e;
    }
    double* spec = w2;      // the divided spectrum
    if (dim == 3) {
        // forward along z with the division: W1 = (Tz W2) / lambda, W2 as nz x (ny nx)
        GemmArgs a{};
        a.a = T[2];
        a.lda = nz;
        a.b = w2;
        a.ldb = pl;
        a.c = w1;
        a.ldc = pl;
        a.m = nz;
        a.n = (int)pl;
        a.k = nz;
        for (int d = 0; d < 3; ++d) a.sig[d] = sg[d];
        a.nx = nx;
        a.three_d = 1;
        a.alpha = cf.alpha;
        a.beta = cf.beta;
        e = gemm(st, EPI_LAMBDA, a, 1);
        if (e != hipSuccess) return e;
        // inverse along z: W2 = Tz^T W1
        GemmArgs c{};
        c.a = Ti[2];
        c.lda = nz;
        c.b = w1;
        c.ldb = pl;
        c.c = w2;
        c.ldc = pl;
        c.m = nz;
        c.n = (int)pl;
        c.k = nz;
        e = gemm(st, EPI_STORE, c, 1);
        if (e != hipSuccess) return e;
        spec = w2;
    }
    // inverse along y: W1[z] = Ty^T spec[z]
    {
        GemmArgs a{};
        a.a = Ti[1];
        a.lda = ny;
        a.b = spec;
        a.ldb = nx;
        a.sb = pl;
        a.c = w1;
        a.ldc = nx;
        a.sc = pl;
        a.m = ny;
        a.n = nx;
        a.k = ny;
        e = gemm(st, EPI_STORE, a, nz);
        if (e != hipSuccess) return e;
    }
    // inverse along x with the update: x[z][j][i] = sum_k W1[z][j][k] Tx[k][i]
    {
        GemmArgs a{};
        a.a = w1;
        a.lda = nx;
        a.sa = pl;
        a.b = T[0];
        a.ldb = nx;
        a.m = ny;
        a.n = nx;
        a.k = nx;
        a.field = field;
        a.ge = ge;
        a.cur = cur;
        a.P = P;
        a.plane = (long)plane;
        a.off = off;
        a.cfl = cf.cfl;
        a.ge_gain = cf.ge_gain;
        a.ge_curl = cf.ge_curl;
        e = gemm(st, EPI_FIELD, a, nz);
    }
    return e;
}

}  // namespace c4m
