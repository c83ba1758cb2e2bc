// c4m_nc.hip -- the non-compact comparison scheme NC (Section 5.2): the Yee
// update of the 2D TM system (maxwell2d) with first derivatives from the
// stencil K4 at a = 0 (eq:K4): on a staggered line
//   D u(x_i) = [27 (u(i+1/2) - u(i-1/2)) - (u(i+3/2) - u(i-3/2))] / (24 h),
// and, where u(i-3/2) or u(i+3/2) is off the grid, the standard one-sided
// row on the four nearest values [-23 u(i-1/2) + 21 u(i+1/2) + 3 u(i+3/2)
// - u(i+5/2)] / (24 h) (mirrored at the far wall).  Two launches a step:
//   Ez += r Z (Dx Hy - Dy Hx)           on the interior nodes,
//   Hx -= (r/Z) Dy Ez,  Hy += (r/Z) Dx Ez   off the walls they are normal to.
// Every thread writes one value; neighbouring threads take neighbouring x,
// so row reads are coalesced and the four rows of a y-stencil come from L2.
#include "c4m_internal.h"

namespace c4m {

// D u (times h) at output k of a line of m inputs u[0], u[s], u[2 s], ...,
// output k midway between inputs k and k + 1.
__device__ __forceinline__ double nc_deriv(const double* __restrict__ u, long s, int k, int m)
{
    if (k >= 1 && k + 2 <= m - 1)
        return (27.0 * (u[(k + 1) * s] - u[k * s]) - (u[(k + 2) * s] - u[(k - 1) * s])) * (1.0 / 24.0);
    if (k == 0) return (-23.0 * u[0] + 21.0 * u[s] + 3.0 * u[2 * s] - u[3 * s]) * (1.0 / 24.0);
    return (23.0 * u[(k + 1) * s] - 21.0 * u[k * s] - 3.0 * u[(k - 1) * s] + u[(k - 2) * s]) * (1.0 / 24.0);
}

constexpr int NC_TX = 64, NC_TY = 4;

// Ez at the interior nodes (i, j), 1 <= i, j <= N-1
__global__ __launch_bounds__(NC_TX * NC_TY) void k_nc_e(double* __restrict__ ez, const double* __restrict__ hx,
                                                      const double* __restrict__ hy, int N, int P, double rz)
{
    const int i = 1 + (int)(blockIdx.x * NC_TX + threadIdx.x % NC_TX);
    const int j = 1 + (int)(blockIdx.y * NC_TY + threadIdx.x / NC_TX);
    if (i > N - 1 || j > N - 1) return;
    const double dxhy = nc_deriv(hy + (size_t)j * P, 1, i - 1, N);      // Hy: half points along x
    const double dyhx = nc_deriv(hx + i, P, j - 1, N);                  // Hx: half points along y
    ez[(size_t)j * P + i] += rz * (dxhy - dyhx);
}

// blockIdx.z 0: Hx at (i, j + 1/2), 1 <= i <= N-1, 0 <= j <= N-1;
//            1: Hy at (i + 1/2, j), 0 <= i <= N-1, 1 <= j <= N-1
__global__ __launch_bounds__(NC_TX * NC_TY) void k_nc_h(const double* __restrict__ ez, double* __restrict__ hx,
                                                      double* __restrict__ hy, int N, int P, double rz_inv)
{
    const int x = (int)(blockIdx.x * NC_TX + threadIdx.x % NC_TX);
    const int y = (int)(blockIdx.y * NC_TY + threadIdx.x / NC_TX);
    if (blockIdx.z == 0) {
        const int i = 1 + x, j = y;
        if (i > N - 1 || j > N - 1) return;
        hx[(size_t)j * P + i] -= rz_inv * nc_deriv(ez + i, P, j, N + 1);
    } else {
        const int i = x, j = 1 + y;
        if (i > N - 1 || j > N - 1) return;
        hy[(size_t)j * P + i] += rz_inv * nc_deriv(ez + (size_t)j * P, 1, i, N + 1);
    }
}

hipError_t launch_nc_e(hipStream_t st, double* ez, const double* hx, const double* hy, int N, int P, double r,
                       double z)
{
    const dim3 grid((N - 1 + NC_TX - 1) / NC_TX, (N - 1 + NC_TY - 1) / NC_TY);
    hipLaunchKernelGGL(k_nc_e, grid, dim3(NC_TX * NC_TY), 0, st, ez, hx, hy, N, P, r * z);
    return hipGetLastError();
}

hipError_t launch_nc_h(hipStream_t st, const double* ez, double* hx, double* hy, int N, int P, double r, double z)
{
    const dim3 grid((N + NC_TX - 1) / NC_TX, (N + NC_TY - 1) / NC_TY, 2);
    hipLaunchKernelGGL(k_nc_h, grid, dim3(NC_TX * NC_TY), 0, st, ez, hx, hy, N, P, r / z);
    return hipGetLastError();
}

}  // namespace c4m
