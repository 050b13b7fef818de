// Standalone grid conversion: y_hat = P y and the three ways of applying P^T
// that Sec. 2.2 ("Grid conversion") compares:
//
// * gather (Eq. 3, the paper's scheme): one thread per deformation node sums
//   omega_x omega_y omega_z z[i] over the index sets of its three axes; every
//   write has one owner;
// * atomic scatter (the earlier GPU scheme): one thread per image point adds
//   its weighted value into the 8 nodes of its cell with atomic additions;
// * red-black slices (the earlier scheme): the image slices of the odd x
//   cells are done in parallel, then those of the even x cells.  A cell's
//   slices reach only the node planes at its two ends, and cells of one
//   parity are two apart, so within a phase no two cells share a node plane;
//   within a cell one thread per (y, z) node sums the slices over its y and
//   z index sets and adds the result to the two node planes (no atomics).
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

// index set of node j along one axis (Eq. 3): the contiguous run of image
// points whose lower node is j - 1 or j, [lo, hi), from the exact integer
// map (no table search)
struct Range {
    int lo, hi;
};
__device__ inline Range omega_range(const Maps& a, int d, int j) {
    return Range{first_at_least(j - 1, a.m[d], a.n[d]), first_at_least(j + 1, a.m[d], a.n[d])};
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
        const Range rx = omega_range(a, 0, jx), ry = omega_range(a, 1, jy),
                    rz = omega_range(a, 2, jz);
        float acc[3] = {0.0f, 0.0f, 0.0f};
        for (int ix = rx.lo; ix < rx.hi; ++ix) {
            const float wx = omega(a, 0, ix, jx);
            for (int iy = ry.lo; iy < ry.hi; ++iy) {
                const float wxy = wx * omega(a, 1, iy, jy);
                for (int iz = rz.lo; iz < rz.hi; ++iz) {
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

// One phase of the red-black scheme: every x cell gx of parity px, one
// thread per (cell, y node, z node).  The thread sums the cell's slices (the
// image points whose lower x node is gx) over its y and z index sets, each
// slice weighted for node plane gx and for gx + 1, and adds both sums to the
// output; no other thread of the phase touches those nodes.
__global__ __launch_bounds__(kThreads) void k_PT_redblack(Maps a, const float* __restrict__ z,
                                                          float* __restrict__ out, int px) {
    const int64_t N = static_cast<int64_t>(a.m[0]) * a.m[1] * a.m[2];
    const int64_t Ny = static_cast<int64_t>(a.n[0]) * a.n[1] * a.n[2];
    const int cells = (a.n[0] - 1 - px + 1) / 2;  // x cells of this parity
    const int64_t nyz = static_cast<int64_t>(a.n[1]) * a.n[2];
    for (int64_t t = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
         t < cells * nyz; t += static_cast<int64_t>(gridDim.x) * kThreads) {
        const int gx = 2 * static_cast<int>(t / nyz) + px;
        const int jy = static_cast<int>((t / a.n[2]) % a.n[1]);
        const int jz = static_cast<int>(t % a.n[2]);
        // the cell's slices: image points with lower x node gx
        const int ilo = first_at_least(gx, a.m[0], a.n[0]);
        const int ihi = first_at_least(gx + 1, a.m[0], a.n[0]);
        const Range ry = omega_range(a, 1, jy), rz = omega_range(a, 2, jz);
        float lo[3] = {0.0f, 0.0f, 0.0f}, hi[3] = {0.0f, 0.0f, 0.0f};
        for (int ix = ilo; ix < ihi; ++ix) {
            const float wx0 = a.w0[0][ix], wx1 = a.w1[0][ix];
            float s[3] = {0.0f, 0.0f, 0.0f};
            for (int iy = ry.lo; iy < ry.hi; ++iy) {
                const float wy = omega(a, 1, iy, jy);
                for (int iz = rz.lo; iz < rz.hi; ++iz) {
                    const float w = wy * omega(a, 2, iz, jz);
                    const int64_t i = (static_cast<int64_t>(ix) * a.m[1] + iy) * a.m[2] + iz;
                    s[0] = fmaf(w, z[i], s[0]);
                    s[1] = fmaf(w, z[N + i], s[1]);
                    s[2] = fmaf(w, z[2 * N + i], s[2]);
                }
            }
            for (int c = 0; c < 3; ++c) {
                lo[c] = fmaf(wx0, s[c], lo[c]);
                hi[c] = fmaf(wx1, s[c], hi[c]);
            }
        }
        const int64_t j = (static_cast<int64_t>(gx) * a.n[1] + jy) * a.n[2] + jz;
        for (int c = 0; c < 3; ++c) {
            out[c * Ny + j] += lo[c];
            out[c * Ny + j + nyz] += hi[c];
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
        // odd x cells, then even ones (the second phase starts after the
        // first on the stream: they share node planes)
        const int64_t nyz = static_cast<int64_t>(n[1]) * n[2];
        for (int px = 1; px >= 0; --px) {
            const int64_t cells = (n[0] - 1 - px + 1) / 2;
            hipLaunchKernelGGL(k_PT_redblack, dim3(blocks_for(cells * nyz)), dim3(kThreads), 0, s,
                               a, z, out, px);
        }
    }
}

}  // namespace ngf
