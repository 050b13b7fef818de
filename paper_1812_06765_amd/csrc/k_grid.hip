// Pyramid, index maps, identity, prolongation, finite check and the final
// fixed-order reduction of an evaluation.
#include "ngf_internal.h"
#include "reduce_body.h"

#include <math.h>

namespace ngf {

namespace {

inline int grid_for(int64_t n, int per_block = kThreads, int cap = 65536) {
    int64_t b = (n + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return static_cast<int>(b);
}

// One pyramid step: coarse voxel = mean of its 8 children, summed in float64
// in the fixed order ((000+001)+(010+011)) + ((100+101)+(110+111)) and
// rounded once to float32.  Contraction is off so the order is exactly this.
__global__ __launch_bounds__(kThreads) void k_downsample(const float* __restrict__ src,
                                                         float* __restrict__ dst, int mx,
                                                         int my, int mz) {
#pragma clang fp contract(off)
    const int cx = mx / 2, cy = my / 2, cz = mz / 2;
    const int64_t n = static_cast<int64_t>(cx) * cy * cz;
    const int64_t sy = mz, sx = static_cast<int64_t>(my) * mz;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int z = static_cast<int>(i % cz);
        const int64_t t = i / cz;
        const int y = static_cast<int>(t % cy);
        const int x = static_cast<int>(t / cy);
        const float* p = src + (2 * x) * sx + (2 * y) * sy + 2 * z;
        const double v000 = p[0], v001 = p[1], v010 = p[sy], v011 = p[sy + 1];
        const double v100 = p[sx], v101 = p[sx + 1], v110 = p[sx + sy], v111 = p[sx + sy + 1];
        const double s = ((v000 + v001) + (v010 + v011)) + ((v100 + v101) + (v110 + v111));
        dst[i] = static_cast<float>(0.125 * s);
    }
}

// Per-axis index map: image point i lies at node coordinate num/den with
// num = (2i+1)(my-1), den = 2m; j0 = num div den, w1 = r/den, w0 = (den-r)/den
// (float64 quotient, correctly rounded, then rounded to float32).
__global__ void k_index_map(int32_t* j0, float* w0, float* w1, int m, int my) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int64_t num = static_cast<int64_t>(2 * i + 1) * (my - 1);
    const int64_t den = 2 * static_cast<int64_t>(m);
    const int64_t j = num / den;
    const int64_t r = num - j * den;
    j0[i] = static_cast<int32_t>(j);
    w1[i] = static_cast<float>(static_cast<double>(r) / static_cast<double>(den));
    w0[i] = static_cast<float>(static_cast<double>(den - r) / static_cast<double>(den));
}

__global__ __launch_bounds__(kThreads) void k_identity(float* y, int nx, int ny, int nz,
                                                       double hx, double hy, double hz) {
    const int64_t n = static_cast<int64_t>(nx) * ny * nz;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int z = static_cast<int>(i % nz);
        const int64_t t = i / nz;
        const int yy = static_cast<int>(t % ny);
        const int x = static_cast<int>(t / ny);
        y[i] = static_cast<float>(x * hx);
        y[n + i] = static_cast<float>(yy * hy);
        y[2 * n + i] = static_cast<float>(z * hz);
    }
}

// Prolongation by the tensor product of 1D operators (fine 2j <- coarse j,
// fine 2j+1 <- mean of coarse j, j+1), averaged along x first, then y, then z.
__global__ __launch_bounds__(kThreads) void k_prolongate(const float* __restrict__ yc,
                                                         float* __restrict__ yf, int cx,
                                                         int cy, int cz) {
#pragma clang fp contract(off)
    const int fx = 2 * cx - 1, fy = 2 * cy - 1, fz = 2 * cz - 1;
    const int64_t nf = static_cast<int64_t>(fx) * fy * fz;
    const int64_t nc = static_cast<int64_t>(cx) * cy * cz;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < 3 * nf;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int c = static_cast<int>(i / nf);
        const int64_t q = i - c * nf;
        const int z = static_cast<int>(q % fz);
        const int64_t t = q / fz;
        const int y = static_cast<int>(t % fy);
        const int x = static_cast<int>(t / fy);
        const int x0 = x >> 1, y0 = y >> 1, z0 = z >> 1;
        const int x1 = x0 + (x & 1), y1 = y0 + (y & 1), z1 = z0 + (z & 1);
        const float* b = yc + c * nc;
        auto at = [&](int a, int bb, int cc) -> double {
            return static_cast<double>(b[(static_cast<int64_t>(a) * cy + bb) * cz + cc]);
        };
        auto ax = [&](int bb, int cc) -> double {
            return (x & 1) ? 0.5 * (at(x0, bb, cc) + at(x1, bb, cc)) : at(x0, bb, cc);
        };
        auto ay = [&](int cc) -> double {
            return (y & 1) ? 0.5 * (ax(y0, cc) + ax(y1, cc)) : ax(y0, cc);
        };
        const double v = (z & 1) ? 0.5 * (ay(z0) + ay(z1)) : ay(z0);
        yf[i] = static_cast<float>(v);
    }
}

__global__ __launch_bounds__(kThreads) void k_check_finite(const float* __restrict__ v,
                                                           int64_t n, int* flag) {
    int bad = 0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        bad |= !isfinite(v[i]);
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

__global__ __launch_bounds__(kThreads) void k_fill(float* p, int64_t n, float v) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

__global__ __launch_bounds__(kThreads) void k_reduce(ReduceArgs a) {
    if (a.gate && *a.gate == kOpNone) return;
    reduce_body(a);
}

// one workgroup per pair
__global__ __launch_bounds__(kThreads) void k_reduce_batch(const ReduceArgs* args) {
    const ReduceArgs& a = args[blockIdx.x];
    if (a.gate && *a.gate == kOpNone) return;
    reduce_body(a);
}

}  // namespace

void launch_downsample(const float* src, float* dst, int mx, int my, int mz, hipStream_t s) {
    const int64_t n = static_cast<int64_t>(mx / 2) * (my / 2) * (mz / 2);
    hipLaunchKernelGGL(k_downsample, dim3(grid_for(n)), dim3(kThreads), 0, s, src, dst, mx, my,
                       mz);
}

void launch_index_map(int32_t* j0, float* w0, float* w1, int m, int my, hipStream_t s) {
    hipLaunchKernelGGL(k_index_map, dim3((m + 255) / 256), dim3(256), 0, s, j0, w0, w1, m, my);
}

void launch_identity(float* y, int nx, int ny, int nz, double hx, double hy, double hz,
                     hipStream_t s) {
    const int64_t n = static_cast<int64_t>(nx) * ny * nz;
    hipLaunchKernelGGL(k_identity, dim3(grid_for(n)), dim3(kThreads), 0, s, y, nx, ny, nz, hx,
                       hy, hz);
}

void launch_prolongate(const float* yc, float* yf, int cx, int cy, int cz, hipStream_t s) {
    const int64_t n = 3LL * (2 * cx - 1) * (2 * cy - 1) * (2 * cz - 1);
    hipLaunchKernelGGL(k_prolongate, dim3(grid_for(n)), dim3(kThreads), 0, s, yc, yf, cx, cy,
                       cz);
}

void launch_check_finite(const float* v, int64_t n, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_check_finite, dim3(grid_for(n, kThreads, 4096)), dim3(kThreads), 0, s,
                       v, n, flag);
}

void launch_fill(float* p, int64_t n, float v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n, kThreads, 8192)), dim3(kThreads), 0, s, p, n, v);
}

void launch_reduce_batch(const ReduceArgs* args, int npairs, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_batch, dim3(npairs), dim3(kThreads), 0, s, args);
}

void launch_reduce(const ReduceArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kThreads), 0, s, a);
}

}  // namespace ngf
