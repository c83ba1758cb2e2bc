// Jacobi-preconditioned conjugate gradients for M Phi = b on one component
// grid (Section 3.2: M is symmetric positive definite; the Conclusions solve
// it by CG in a few iterations).  Dot products are reduced on the device in a
// fixed order (wave shuffles, then the LDS, then one partial per workgroup,
// summed by the last workgroup to finish), so results do not depend on
// scheduling.  The host queues a fixed number of iterations; once the
// residual target is met every later kernel of the solve returns at once.
#include <hip/hip_runtime.h>

#include "c4m_internal.h"

namespace c4m {

namespace {

constexpr int PCG_THREADS = 256;
constexpr int PCG_MAX_BLOCKS = 2048;   // grid cap: threads stride over the cells

// Unknown (i, j, k) number e of the box g (x fastest).
__device__ __forceinline__ void pcg_cell(const UGrid& g, long e, int& i, int& j, int& k)
{
    const int nx = g.hi[0] - g.lo[0], ny = g.hi[1] - g.lo[1];
    i = g.lo[0] + (int)(e % nx);
    const long rest = e / nx;
    j = g.lo[1] + (int)(rest % ny);
    k = g.lo[2] + (int)(rest / ny);
}

__device__ __forceinline__ long pcg_cells(const UGrid& g)
{
    return (long)(g.hi[0] - g.lo[0]) * (g.hi[1] - g.lo[1]) * (g.hi[2] - g.lo[2]);
}

// Index of a stencil neighbour: Dirichlet outside the unknowns -> -1 (value
// zero), Neumann -> mirrored back onto the edge unknown (even ghost).
__device__ __forceinline__ long nb_index(const PcgArgs& a, int i, int j, int k)
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

// Calls f(index, weight) for every stencil neighbour of L9 (weights x6):
// 2D: 4 on edges, 1 on corners; 3D: 2 on faces, 1 on edges.
template <int DIM, class F>
__device__ __forceinline__ void for_neighbours(const PcgArgs& a, int i, int j, int k, F&& f)
{
    if (DIM == 2) {
        f(nb_index(a, i - 1, j, k), 4.0);
        f(nb_index(a, i + 1, j, k), 4.0);
        f(nb_index(a, i, j - 1, k), 4.0);
        f(nb_index(a, i, j + 1, k), 4.0);
        f(nb_index(a, i - 1, j - 1, k), 1.0);
        f(nb_index(a, i + 1, j - 1, k), 1.0);
        f(nb_index(a, i - 1, j + 1, k), 1.0);
        f(nb_index(a, i + 1, j + 1, k), 1.0);
    } else {
        f(nb_index(a, i - 1, j, k), 2.0);
        f(nb_index(a, i + 1, j, k), 2.0);
        f(nb_index(a, i, j - 1, k), 2.0);
        f(nb_index(a, i, j + 1, k), 2.0);
        f(nb_index(a, i, j, k - 1), 2.0);
        f(nb_index(a, i, j, k + 1), 2.0);
        for (int s = -1; s <= 1; s += 2)
            for (int t = -1; t <= 1; t += 2) {
                f(nb_index(a, i + s, j + t, k), 1.0);
                f(nb_index(a, i, j + s, k + t), 1.0);
                f(nb_index(a, i + s, j, k + t), 1.0);
            }
    }
}

// Diagonal of M at an unknown.  A neighbour lands on the cell itself when
// every axis it steps along is a Neumann axis at that edge (even ghost); its
// weight then adds to the centre: alpha - beta (centre + those weights) / 6.
template <int DIM>
__device__ __forceinline__ double m_diag(const PcgArgs& a, int i, int j, int k)
{
    const int q[3] = {i, j, k};
    double lo[3], hi[3];                  // 1 if the step -1 / +1 along d lands on the cell
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lo[d] = a.g.neumann[d] && q[d] == a.g.lo[d] ? 1.0 : 0.0;
        hi[d] = a.g.neumann[d] && q[d] == a.g.hi[d] - 1 ? 1.0 : 0.0;
    }
    double w;
    if (DIM == 2) {
        const double sx = lo[0] + hi[0], sy = lo[1] + hi[1];
        w = -20.0 + 4.0 * (sx + sy) + sx * sy;
    } else {
        const double s0 = lo[0] + hi[0], s1 = lo[1] + hi[1], s2 = lo[2] + hi[2];
        w = -24.0 + 2.0 * (s0 + s1 + s2) + s0 * s1 + s1 * s2 + s0 * s2;
    }
    return fma(-a.beta, w * (1.0 / 6.0), a.alpha);
}

// Block sum of one value per thread (wave shuffles, then the LDS); the total
// is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* lds)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < PCG_THREADS / 64; ++w) s += lds[w];
    __syncthreads();
    return s;
}

// Store this workgroup's NV partial sums; returns true in every thread of the
// last workgroup to finish, which then sees all partials.
template <int NV>
__device__ __forceinline__ bool publish_partials(const PcgArgs& a, const double (&v)[NV], int* flag)
{
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) a.part[(size_t)q * a.nparts + blockIdx.x] = v[q];
        __threadfence();
        const int done = atomicAdd(&a.st->arrived, 1);
        *flag = done == (int)gridDim.x - 1;
    }
    __syncthreads();
    const bool last = *flag != 0;
    if (last) __threadfence();
    return last;
}

// Sum of partial array q over all workgroups in a fixed order (strided per
// thread, then the block tree), valid in thread 0 of the last workgroup.
__device__ __forceinline__ double total(const PcgArgs& a, int q, double* lds)
{
    double s = 0.0;
    const double* p = a.part + (size_t)q * a.nparts;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += PCG_THREADS)
        s += __hip_atomic_load(p + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return block_sum(s, lds);
}

// Calls f(o, i, j, k) for this thread's unknowns: a grid-stride sweep in a
// fixed order, so every partial sum is formed the same way on every run.
template <class F>
__device__ __forceinline__ void for_cells(const PcgArgs& a, F&& f)
{
    const long n = pcg_cells(a.g);
    for (long e = (long)blockIdx.x * PCG_THREADS + threadIdx.x; e < n; e += (long)gridDim.x * PCG_THREADS) {
        int i, j, k;
        pcg_cell(a.g, e, i, j, k);
        f((long)k * (long)a.plane + (long)j * a.P + i, i, j, k);
    }
}

// x = 0, r = b (in place), p_old = 0, z = r / diag; rz = <r, z>, bb = <b, b>.
template <int DIM>
__global__ __launch_bounds__(PCG_THREADS) void k_pcg_init(PcgArgs a)
{
    __shared__ double lds[PCG_THREADS / 64];
    __shared__ int flag;
    double v[2] = {0.0, 0.0};
    for_cells(a, [&](long o, int i, int j, int k) {
        const double rr = a.r[o];
        const double di = 1.0 / m_diag<DIM>(a, i, j, k);
        a.dinv[o] = di;
        a.z[o] = rr * di;
        a.x[o] = 0.0;
        a.p[0][o] = 0.0;
        v[0] += rr * rr * di;
        v[1] += rr * rr;
    });
    double s[2];
    s[0] = block_sum(v[0], lds);
    s[1] = block_sum(v[1], lds);
    if (!publish_partials<2>(a, s, &flag)) return;
    const double rz = total(a, 0, lds);
    const double bb = total(a, 1, lds);
    if (threadIdx.x == 0) {
        PcgState* st = a.st;
        st->arrived = 0;
        st->rz = rz;
        st->bb = bb;
        st->beta = 0.0;
        st->rr = bb;
        st->iters = 0;
        st->done = bb == 0.0 ? 1 : 0;
    }
}

// p_new = z + beta p_old (at the cell and, on the fly, at its neighbours),
// q = M p_new; partial <p_new, q>.  The last workgroup sets alpha.
template <int DIM>
__global__ __launch_bounds__(PCG_THREADS) void k_pcg_mp(PcgArgs a, int it)
{
    if (a.st->done) return;
    __shared__ double lds[PCG_THREADS / 64];
    __shared__ int flag;
    const double* __restrict__ pold = a.p[it & 1];
    double* __restrict__ pnew = a.p[(it & 1) ^ 1];
    const double beta = a.st->beta;
    double v[1] = {0.0};
    for_cells(a, [&](long o, int i, int j, int k) {
        auto pval = [&](long q) { return fma(beta, pold[q], a.z[q]); };
        const double pc = pval(o);
        double side = 0.0;
        for_neighbours<DIM>(a, i, j, k, [&](long q, double wt) {
            if (q >= 0) side += wt * pval(q);
        });
        const double l9 = (side + (DIM == 2 ? -20.0 : -24.0) * pc) * (1.0 / 6.0);
        const double qv = fma(a.alpha, pc, -a.beta * l9);
        pnew[o] = pc;
        a.q[o] = qv;
        v[0] += pc * qv;
    });
    double s[1];
    s[0] = block_sum(v[0], lds);
    if (!publish_partials<1>(a, s, &flag)) return;
    const double pq = total(a, 0, lds);
    if (threadIdx.x == 0) {
        a.st->arrived = 0;
        a.st->alpha = pq > 0.0 ? a.st->rz / pq : 0.0;
    }
}

// x += alpha p, r -= alpha q, z = r / diag; partials <r, z>, <r, r>.  The
// last workgroup sets beta, the convergence flag and the iteration count.
template <int DIM>
__global__ __launch_bounds__(PCG_THREADS) void k_pcg_update(PcgArgs a, int it)
{
    if (a.st->done) return;
    __shared__ double lds[PCG_THREADS / 64];
    __shared__ int flag;
    const double* __restrict__ pc = a.p[(it & 1) ^ 1];
    const double alpha = a.st->alpha;
    double v[2] = {0.0, 0.0};
    for_cells(a, [&](long o, int, int, int) {
        a.x[o] = fma(alpha, pc[o], a.x[o]);
        const double rn = fma(-alpha, a.q[o], a.r[o]);
        const double zn = rn * a.dinv[o];
        a.r[o] = rn;
        a.z[o] = zn;
        v[0] += rn * zn;
        v[1] += rn * rn;
    });
    double s[2];
    s[0] = block_sum(v[0], lds);
    s[1] = block_sum(v[1], lds);
    if (!publish_partials<2>(a, s, &flag)) return;
    const double rz = total(a, 0, lds);
    const double rr = total(a, 1, lds);
    if (threadIdx.x == 0) {
        PcgState* st = a.st;
        st->arrived = 0;
        st->beta = st->rz > 0.0 ? rz / st->rz : 0.0;
        st->rz = rz;
        st->rr = rr;
        st->iters = it + 1;
        if (rr <= a.rtol2 * st->bb) st->done = 1;
    }
}

// field += cfl x; with the carried Laplacian of E also
// G_E += (1 + 4/r^2) dE - (2/r) Z c.  Records the solve's statistics.
__global__ __launch_bounds__(PCG_THREADS) void k_pcg_final(PcgArgs a, double* field, double* ge, const double* cur,
                                                            Coef cf)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        PcgState* st = a.st;
        st->last_iters = st->iters;
        st->max_iters = st->iters > st->max_iters ? st->iters : st->max_iters;
        st->last_rel = st->bb > 0.0 ? sqrt(st->rr / st->bb) : 0.0;
        if (!st->done) st->noconv = 1;
    }
    for_cells(a, [&](long o, int, int, int) {
        const double de = cf.cfl * a.x[o];
        field[o] += de;
        if (ge) ge[o] += fma(cf.ge_gain, de, -cf.ge_curl * cur[o]);
    });
}

}  // namespace

size_t pcg_partials(const UGrid& g)
{
    const long cells = (long)(g.hi[0] - g.lo[0]) * (g.hi[1] - g.lo[1]) * (g.hi[2] - g.lo[2]);
    const long blocks = (cells + PCG_THREADS - 1) / PCG_THREADS;
    return (size_t)(blocks < PCG_MAX_BLOCKS ? blocks : PCG_MAX_BLOCKS);
}

// One solve M x = b (b in a.r, overwritten) of at most max_iter iterations,
// then field += cfl x (and the G_E update when ge is given).
hipError_t launch_pcg(hipStream_t st, int dim, PcgArgs a, int max_iter, double* field, double* ge,
                      const double* cur, const Coef& cf)
{
    const dim3 grid((unsigned)pcg_partials(a.g));
    a.nparts = grid.x;
    if (dim == 2) {
        hipLaunchKernelGGL(k_pcg_init<2>, grid, dim3(PCG_THREADS), 0, st, a);
        for (int it = 0; it < max_iter; ++it) {
            hipLaunchKernelGGL(k_pcg_mp<2>, grid, dim3(PCG_THREADS), 0, st, a, it);
            hipLaunchKernelGGL(k_pcg_update<2>, grid, dim3(PCG_THREADS), 0, st, a, it);
        }
    } else {
        hipLaunchKernelGGL(k_pcg_init<3>, grid, dim3(PCG_THREADS), 0, st, a);
        for (int it = 0; it < max_iter; ++it) {
            hipLaunchKernelGGL(k_pcg_mp<3>, grid, dim3(PCG_THREADS), 0, st, a, it);
            hipLaunchKernelGGL(k_pcg_update<3>, grid, dim3(PCG_THREADS), 0, st, a, it);
        }
    }
    hipLaunchKernelGGL(k_pcg_final, grid, dim3(PCG_THREADS), 0, st, a, field, ge, cur, cf);
    return hipGetLastError();
}

}  // namespace c4m
