// c4m_kernels_common.hip -- elementwise kernels shared by the 2D and 3D
// paths: wall conditions on set, conversions between the carried Laplacian
// l = h^2 Delta E and the stored G_E = alpha E + l/12, and the finite check.
#include "c4m_internal.h"

namespace c4m {

__device__ __forceinline__ bool on_node_wall(const Box& bx, int i, int j, int k)
{
    const int q[3] = {i, j, k};
#pragma unroll
    for (int d = 0; d < 3; ++d)
        if (bx.active[d] && !bx.half[d] && (q[d] == 0 || q[d] == bx.n[d] - 1)) return true;
    return false;
}

__global__ void k_zero_walls(double* a, Box bx, int P, size_t plane)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    const int k = blockIdx.z;
    if (i >= bx.n[0]) return;
    if (on_node_wall(bx, i, j, k)) a[k * plane + (size_t)j * P + i] = 0.0;
}

// mode 0: ge = alpha e + l / 12   (array `a` holds l on entry, G_E on exit)
// mode 1: out = 12 (ge - alpha e) (array `a` holds G_E; l written to `out`)
// mode 2: a = alpha e + L5 e / 12 (G_E from E alone; l = L5 E, the
//         second-order Laplacian with even ghosts along the half axis)
__global__ void k_lap_convert(double* a, const double* e, double* out, Box bx, int P, size_t plane,
                              double alpha, int mode)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    const int k = blockIdx.z;
    if (i >= bx.n[0]) return;
    const size_t o = k * plane + (size_t)j * P + i;
    if (mode == 0) {
        a[o] = on_node_wall(bx, i, j, k) ? 0.0 : fma(alpha, e[o], a[o] * (1.0 / 12.0));
    } else if (mode == 1) {
        out[o] = on_node_wall(bx, i, j, k) ? 0.0 : 12.0 * (a[o] - alpha * e[o]);
    } else {
        if (on_node_wall(bx, i, j, k)) {
            a[o] = 0.0;
            return;
        }
        const int q[3] = {i, j, k};
        const size_t st[3] = {1, (size_t)P, plane};
        double lap = 0.0;
        for (int d = 0; d < 3; ++d) {
            if (!bx.active[d]) continue;
            const size_t om = (q[d] == 0) ? o : o - st[d];            // even ghost (half axis)
            const size_t op = (q[d] == bx.n[d] - 1) ? o : o + st[d];
            lap += e[om] + e[op] - 2.0 * e[o];
        }
        a[o] = fma(alpha, e[o], lap * (1.0 / 12.0));
    }
}

// Count of non-finite entries (atomic add into one int).
__global__ void k_count_nonfinite(const double* a, Box bx, int P, size_t plane, int* count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    const int k = blockIdx.z;
    bool bad = false;
    if (i < bx.n[0]) bad = !isfinite(a[k * plane + (size_t)j * P + i]);
    const unsigned long long m = __ballot(bad);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(count, __popcll(m));
}

static dim3 box_grid(const Box& bx) { return dim3((bx.n[0] + 255) / 256, bx.n[1], bx.n[2]); }

hipError_t launch_zero_walls(hipStream_t st, double* a, const Box& bx, int P, size_t plane)
{
    hipLaunchKernelGGL(k_zero_walls, box_grid(bx), dim3(256), 0, st, a, bx, P, plane);
    return hipGetLastError();
}

hipError_t launch_lap_convert(hipStream_t st, double* a, const double* e, double* out, const Box& bx,
                              int P, size_t plane, double alpha, int mode)
{
    hipLaunchKernelGGL(k_lap_convert, box_grid(bx), dim3(256), 0, st, a, e, out, bx, P, plane, alpha,
                       mode);
    return hipGetLastError();
}

hipError_t launch_count_nonfinite(hipStream_t st, const double* a, const Box& bx, int P, size_t plane,
                                  int* count)
{
    hipLaunchKernelGGL(k_count_nonfinite, box_grid(bx), dim3(256), 0, st, a, bx, P, plane, count);
    return hipGetLastError();
}

}  // namespace c4m
