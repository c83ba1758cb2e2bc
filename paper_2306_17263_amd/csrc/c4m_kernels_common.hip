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

// Largest magnitude over the array (out[0]) and over its node walls
// (out[1]), as bit patterns of non-negative doubles (which order like the
// values) combined with atomicMax; NaN counts as infinity.
__global__ void k_wall_max(const double* a, Box bx, int P, size_t plane, unsigned long long* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    const int k = blockIdx.z;
    double v = 0.0, w = 0.0;
    if (i < bx.n[0]) {
        v = fabs(a[k * plane + (size_t)j * P + i]);
        v = isnan(v) ? INFINITY : v;
        w = on_node_wall(bx, i, j, k) ? v : 0.0;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        v = fmax(v, __shfl_xor(v, off));
        w = fmax(w, __shfl_xor(w, off));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(out, (unsigned long long)__double_as_longlong(v));
        atomicMax(out + 1, (unsigned long long)__double_as_longlong(w));
    }
}

// Scatter a contiguous wall plane (the box without `axis`, remaining axes
// in (z, y, x) order, x fastest) into index `at` along `axis`.
__global__ void k_put_plane(double* a, const double* vals, Box bx, int axis, int at, int P, size_t plane)
{
    const int u = axis == 0 ? 1 : 0;          // faster remaining axis
    const int v = axis == 2 ? 1 : 2;          // slower remaining axis
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= bx.n[u] * bx.n[v]) return;
    int q[3];
    q[axis] = at;
    q[u] = e % bx.n[u];
    q[v] = e / bx.n[u];
    a[q[2] * plane + (size_t)q[1] * P + q[0]] = vals[e];
}

// h^2 Delta_h a (sum of second differences; even ghosts along half axes)
// at point o of box bx, valid off the node walls
__device__ __forceinline__ double lap5_at(const double* a, const Box& bx, int P, size_t plane, int i, int j, int k)
{
    const int q[3] = {i, j, k};
    const size_t st[3] = {1, (size_t)P, plane};
    const size_t o = k * plane + (size_t)j * P + i;
    double lap = 0.0;
    for (int d = 0; d < 3; ++d) {
        if (!bx.active[d]) continue;
        const size_t om = (q[d] == 0) ? o : o - st[d];
        const size_t op = (q[d] == bx.n[d] - 1) ? o : o + st[d];
        lap += a[om] - 2.0 * a[o] + a[op];
    }
    return lap;
}

// Taylor start of H: out = h^2 Delta_h a off the node walls, 0 on them
__global__ void k_taylor_lap(const double* a, double* out, Box bx, int P, size_t plane)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    const int k = blockIdx.z;
    if (i >= bx.n[0]) return;
    out[k * plane + (size_t)j * P + i] = on_node_wall(bx, i, j, k) ? 0.0 : lap5_at(a, bx, P, plane, i, j, k);
}

// h += c[0] cu + c[1] lh + c[2] h^2 Delta_h cu + c[3] h^2 Delta_h lh off the node walls
__global__ void k_taylor_combine(double* h, const double* cu, const double* lh, Box bx, int P, size_t plane,
                                 double c0, double c1, double c2, double c3)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    const int k = blockIdx.z;
    if (i >= bx.n[0] || on_node_wall(bx, i, j, k)) return;
    const size_t o = k * plane + (size_t)j * P + i;
    h[o] += c0 * cu[o] + c1 * lh[o] + c2 * lap5_at(cu, bx, P, plane, i, j, k) + c3 * lap5_at(lh, bx, P, plane, i, j, k);
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

hipError_t launch_wall_max(hipStream_t st, const double* a, const Box& bx, int P, size_t plane,
                           unsigned long long* out)
{
    hipLaunchKernelGGL(k_wall_max, box_grid(bx), dim3(256), 0, st, a, bx, P, plane, out);
    return hipGetLastError();
}

hipError_t launch_put_plane(hipStream_t st, double* a, const double* vals, const Box& bx, int axis, int at,
                            int P, size_t plane)
{
    const int cnt = bx.n[0] * bx.n[1] * bx.n[2] / bx.n[axis];
    hipLaunchKernelGGL(k_put_plane, dim3((cnt + 255) / 256), dim3(256), 0, st, a, vals, bx, axis, at, P, plane);
    return hipGetLastError();
}

hipError_t launch_taylor_lap(hipStream_t st, const double* a, double* out, const Box& bx, int P, size_t plane)
{
    hipLaunchKernelGGL(k_taylor_lap, box_grid(bx), dim3(256), 0, st, a, out, bx, P, plane);
    return hipGetLastError();
}

hipError_t launch_taylor_combine(hipStream_t st, double* h, const double* cu, const double* lh, const Box& bx, int P,
                                 size_t plane, const double c[4])
{
    hipLaunchKernelGGL(k_taylor_combine, box_grid(bx), dim3(256), 0, st, h, cu, lh, bx, P, plane, c[0], c[1], c[2],
                       c[3]);
    return hipGetLastError();
}

hipError_t launch_count_nonfinite(hipStream_t st, const double* a, const Box& bx, int P, size_t plane,
                                  int* count)
{
    hipLaunchKernelGGL(k_count_nonfinite, box_grid(bx), dim3(256), 0, st, a, bx, P, plane, count);
    return hipGetLastError();
}

}  // namespace c4m
