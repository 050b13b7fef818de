// Standalone grid conversion: y_hat = P y and the three ways of applying P^T
// that Sec. 2.2 ("Grid conversion") compares:
//
// * gather (Eq. 3, the paper's scheme): one thread per deformation node sums
//   omega_x omega_y omega_z z[i] over the index sets of its three axes; every
//   write has one owner;
// * atomic scatter (the earlier GPU scheme): one thread per image point adds
//   its weighted value into the 8 nodes of its cell with atomic additions;
// * red-black slices (the earlier CPU scheme): image points are grouped by
//   their x and y cell; groups whose cells are two apart never touch the same
//   node, so four colour phases run one thread per group, each thread
//   scattering its group serially without atomics.
//
// All three compute the same sums (in different orders).  These operators
// are for measurement and testing; the evaluation itself fuses P into the
// warp and P^T into the image and node passes.
#include "ngf_internal.h"

namespace ngf {

namespace {

struct Maps {
    const int32_t* j0[3];
    const float* w0[3];
    const float* w1[3];
    int m[3];
    int n[3];
};

// y_hat = P y (float64 accumulation, float32 result); y, yhat component-major
__global__ __launch_bounds__(kThreads) void k_apply_P(Maps a, const float* __restrict__ y,
                                                      float* __restrict__ yh) {
    const int64_t N = static_cast<int64_t>(a.m[0]) * a.m[1] * a.m[2];
    const int64_t Ny = static_cast<int64_t>(a.n[0]) * a.n[1] * a.n[2];
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < N;
         i += static_cast<int64_t>(gridDim.x) * kThreads) {
        const int iz = static_cast<int>(i % a.m[2]);
        const int iy = static_cast<int>((i / a.m[2]) % a.m[1]);
        const int ix = static_cast<int>(i / (static_cast<int64_t>(a.m[2]) * a.m[1]));
        const int jx = a.j0[0][ix], jy = a.j0[1][iy], jz = a.j0[2][iz];
        const double wx[2] = {a.w0[0][ix], a.w1[0][ix]};
        const double wy[2] = {a.w0[1][iy], a.w1[1][iy]};
        const double wz[2] = {a.w0[2][iz], a.w1[2][iz]};
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int p = 0; p < 2; ++p)
                for (int q = 0; q < 2; ++q)
                    for (int r = 0; r < 2; ++r)
                        s += wx[p] * wy[q] * wz[r] *
                             static_cast<double>(
                                 y[c * Ny + ((jx + p) * static_cast<int64_t>(a.n[1]) + jy + q) *
                                                a.n[2] + jz + r]);
            yh[c * N + i] = static_cast<float>(s);
        }
    }
}

// weight of image index i for node j along one axis (0 outside the index set)
__device__ inline float omega(const Maps& a, int d, int i, int j) {
    const int j0 = a.j0[d][i];
    return j0 == j ? a.w0[d][i] : (j0 + 1 == j ? a.w1[d][i] : 0.0f);
}

// first image index of node j's index set along one axis (the set is the
// contiguous run of image points whose cell touches the node)
__device__ inline int omega_lo(const Maps& a, int d, int j) {
    int lo = 0, hi = a.m[d];  // smallest i with j0[i] + 1 >= j
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a.j0[d][mid] + 1 >= j)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

__global__ __launch_bounds__(kThreads) void k_PT_gather(Maps a, const float* __restrict__ z,
                                                        float* __restrict__ out) {
    const int64_t N = static_cast<int64_t>(a.m[0]) * a.m[1] * a.m[2];
    const int64_t Ny = static_cast<int64_t>(a.n[0]) * a.n[1] * a.n[2];
    for (int64_t j = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; j < Ny;
         j += static_cast<int64_t>(gridDim.x) * kThreads) {
        const int jz = static_cast<int>(j % a.n[2]);
        const int jy = static_cast<int>((j / a.n[2]) % a.n[1]);
        const int jx = static_cast<int>(j / (static_cast<int64_t>(a.n[2]) * a.n[1]));
        const int lx = omega_lo(a, 0, jx), ly = omega_lo(a, 1, jy), lz = omega_lo(a, 2, jz);
        float acc[3] = {0.0f, 0.0f, 0.0f};
        for (int ix = lx; ix < a.m[0] && a.j0[0][ix] <= jx; ++ix) {
            const float wx = omega(a, 0, ix, jx);
            for (int iy = ly; iy < a.m[1] && a.j0[1][iy] <= jy; ++iy) {
                const float wxy = wx * omega(a, 1, iy, jy);
                for (int iz = lz; iz < a.m[2] && a.j0[2][iz] <= jz; ++iz) {
                    const float w = wxy * omega(a, 2, iz, jz);
                    const int64_t i = (static_cast<int64_t>(ix) * a.m[1] + iy) * a.m[2] + iz;
                    acc[0] = fmaf(w, z[i], acc[0]);
                    acc[1] = fmaf(w, z[N + i], acc[1]);
                    acc[2] = fmaf(w, z[2 * N + i], acc[2]);
                }
            }
        }
        out[j] = acc[0];
        out[Ny + j] = acc[1];
        out[2 * Ny + j] = acc[2];
    }
}

__global__ __launch_bounds__(kThreads) void k_PT_atomic(Maps a, const float* __restrict__ z,
                                                        float* __restrict__ out) {
    const int64_t N = static_cast<int64_t>(a.m[0]) * a.m[1] * a.m[2];
    const int64_t Ny = static_cast<int64_t>(a.n[0]) * a.n[1] * a.n[2];
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < N;
         i += static_cast<int64_t>(gridDim.x) * kThreads) {
        const int iz = static_cast<int>(i % a.m[2]);
        const int iy = static_cast<int>((i / a.m[2]) % a.m[1]);
        const int ix = static_cast<int>(i / (static_cast<int64_t>(a.m[2]) * a.m[1]));
        const int jx = a.j0[0][ix], jy = a.j0[1][iy], jz = a.j0[2][iz];
        const float wx[2] = {a.w0[0][ix], a.w1[0][ix]};
        const float wy[2] = {a.w0[1][iy], a.w1[1][iy]};
        const float wz[2] = {a.w0[2][iz], a.w1[2][iz]};
        const float v[3] = {z[i], z[N + i], z[2 * N + i]};
        for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q)
                for (int r = 0; r < 2; ++r) {
                    const float w = wx[p] * wy[q] * wz[r];
                    const int64_t j =
                        ((jx + p) * static_cast<int64_t>(a.n[1]) + jy + q) * a.n[2] + jz + r;
                    atomicAdd(out + j, w * v[0]);
                    atomicAdd(out + Ny + j, w * v[1]);
                    atomicAdd(out + 2 * Ny + j, w * v[2]);
                }
    }
}

// One colour phase of the red-black scheme: thread (gx, gy) with cell
// parities (px, py) scatters every image point whose x cell is gx and y cell
// is gy, serially, into nodes {gx, gx+1} x {gy, gy+1} x all z.
__global__ __launch_bounds__(kThreads) void k_PT_redblack(Maps a, const float* __restrict__ z,
                                                          float* __restrict__ out, int px,
                                                          int py, int cells_x, int cells_y) {
    const int64_t N = static_cast<int64_t>(a.m[0]) * a.m[1] * a.m[2];
    const int64_t Ny = static_cast<int64_t>(a.n[0]) * a.n[1] * a.n[2];
    const int hx = (cells_x - px + 1) / 2, hy = (cells_y - py + 1) / 2;
    const int t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= hx * hy) return;
    const int gx = 2 * (t / hy) + px, gy = 2 * (t % hy) + py;
    const int lx = omega_lo(a, 0, gx), ly = omega_lo(a, 1, gy);
    for (int ix = lx; ix < a.m[0] && a.j0[0][ix] <= gx; ++ix) {
        if (a.j0[0][ix] != gx) continue;
        for (int iy = ly; iy < a.m[1] && a.j0[1][iy] <= gy; ++iy) {
            if (a.j0[1][iy] != gy) continue;
            const float wx[2] = {a.w0[0][ix], a.w1[0][ix]};
            const float wy[2] = {a.w0[1][iy], a.w1[1][iy]};
            for (int iz = 0; iz < a.m[2]; ++iz) {
                const int jz = a.j0[2][iz];
                const float wz[2] = {a.w0[2][iz], a.w1[2][iz]};
                const int64_t i = (static_cast<int64_t>(ix) * a.m[1] + iy) * a.m[2] + iz;
                for (int p = 0; p < 2; ++p)
                    for (int q = 0; q < 2; ++q)
                        for (int r = 0; r < 2; ++r) {
                            const float w = wx[p] * wy[q] * wz[r];
                            const int64_t j =
                                ((gx + p) * static_cast<int64_t>(a.n[1]) + gy + q) * a.n[2] +
                                jz + r;
                            out[j] += w * z[i];
                            out[Ny + j] += w * z[N + i];
                            out[2 * Ny + j] += w * z[2 * N + i];
                        }
            }
        }
    }
}

Maps make_maps(const int32_t* const j0[3], const float* const w0[3], const float* const w1[3],
               const int m[3], const int n[3]) {
    Maps a{};
    for (int d = 0; d < 3; ++d) {
        a.j0[d] = j0[d];
        a.w0[d] = w0[d];
        a.w1[d] = w1[d];
        a.m[d] = m[d];
        a.n[d] = n[d];
    }
    return a;
}

int blocks_for(int64_t n) {
    int64_t b = (n + kThreads - 1) / kThreads;
    return static_cast<int>(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

}  // namespace

void launch_apply_P(const int32_t* const j0[3], const float* const w0[3],
                    const float* const w1[3], const int m[3], const int n[3], const float* y,
                    float* yh, hipStream_t s) {
    const Maps a = make_maps(j0, w0, w1, m, n);
    const int64_t N = static_cast<int64_t>(m[0]) * m[1] * m[2];
    hipLaunchKernelGGL(k_apply_P, dim3(blocks_for(N)), dim3(kThreads), 0, s, a, y, yh);
}

// scheme: 0 gather, 1 atomic scatter, 2 red-black.  `out` must be zeroed by
// the caller for schemes 1 and 2.
void launch_apply_PT(const int32_t* const j0[3], const float* const w0[3],
                     const float* const w1[3], const int m[3], const int n[3], const float* z,
                     float* out, int scheme, hipStream_t s) {
    const Maps a = make_maps(j0, w0, w1, m, n);
    const int64_t N = static_cast<int64_t>(m[0]) * m[1] * m[2];
    const int64_t Ny = static_cast<int64_t>(n[0]) * n[1] * n[2];
    if (scheme == 0) {
        hipLaunchKernelGGL(k_PT_gather, dim3(blocks_for(Ny)), dim3(kThreads), 0, s, a, z, out);
    } else if (scheme == 1) {
        hipLaunchKernelGGL(k_PT_atomic, dim3(blocks_for(N)), dim3(kThreads), 0, s, a, z, out);
    } else {
        // cells along x and y: node indices 0 .. n-2 (a cell joins nodes j, j+1)
        const int cx = n[0] - 1, cy = n[1] - 1;
        for (int px = 0; px < 2; ++px)
            for (int py = 0; py < 2; ++py) {
                const int hx = (cx - px + 1) / 2, hy = (cy - py + 1) / 2;
                const int threads = hx * hy;
                hipLaunchKernelGGL(k_PT_redblack, dim3((threads + kThreads - 1) / kThreads),
                                   dim3(kThreads), 0, s, a, z, out, px, py, cx, cy);
            }
    }
}

}  // namespace ngf
