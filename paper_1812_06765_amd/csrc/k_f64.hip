// Float64 evaluation of J and grad J (Eq. 1-3), for the precision study.
//
// The production evaluation keeps the bulk arithmetic in float32 (Sec. 2.2
// computes in single precision) and fuses every image-grid step into one
// pass.  This file computes the same objective with every value in float64,
// as plain, unfused kernels over the image and node grids, so that the
// effect of float32 can be measured on the device against a float64 run of
// the same method:
//
//   k64_warp     P y (trilinear, exact rational weights), the warp T(P y) and
//                its derivative with respect to y_hat           per voxel
//   k64_ngf      central differences of T_y and R, the NGF terms (Eq. 2),
//                v = dD/d(grad T_y), partial sums of 1 - r^2     per voxel
//   k64_adjoint  e = sum_d G_d^T v_d and z = e dT_y/dy_hat      per voxel
//   k64_lap      A u for u = y - X (seven-point, replicated ghost nodes),
//                partial sums of (A u)^2                          per node
//   k64_node     P^T z (Eq. 3, gather over the index sets) plus
//                alpha hbar^y A (A u)                             per node
//   k64_reduce   D, S and J from the partial sums in a fixed order
//
// Intermediates live in one float64 scratch buffer of the context:
// T_y (N), dT_y/dy_hat (3N, overwritten by z), v (3N), A u (3 N^y) and the
// partial sums.  Every reduction has a fixed order (fixed grid, fixed tree),
// so equal inputs give equal outputs.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "../../include/ngfreg.h"
#include "ngf_ctx.h"
#include "ngf_internal.h"

namespace {

constexpr int kT = 256;        // threads per workgroup
constexpr int kBlocks = 1024;  // fixed grid of the reducing kernels

struct Grid64 {
    int m[3], my[3];
    double h[3], hy[3];
    int64_t n, ny;
};

__device__ inline double block_sum(double v, double* s) {
    s[threadIdx.x] = v;
    __syncthreads();
    for (int k = kT / 2; k > 0; k >>= 1) {
        if (static_cast<int>(threadIdx.x) < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    return s[0];
}

// Index map of one axis (Sec. 2.2, "Grid conversion"): image point i lies at
// node coordinate num/den, num = (2i+1)(m^y-1), den = 2m; node j0 = num div
// den takes weight (den - r)/den and node j0+1 weight r/den, r = num mod den.
__device__ inline void index_map(int i, int m, int my, int& j0, double& w0, double& w1) {
    const int64_t num = (2 * static_cast<int64_t>(i) + 1) * (my - 1);
    const int64_t den = 2 * static_cast<int64_t>(m);
    const int64_t q = num / den;
    const int64_t r = num - q * den;
    j0 = static_cast<int>(q);
    w1 = static_cast<double>(r) / static_cast<double>(den);
    w0 = static_cast<double>(den - r) / static_cast<double>(den);
}

__device__ inline void voxel(int64_t n, const Grid64& g, int& ix, int& iy, int& iz) {
    iz = static_cast<int>(n % g.m[2]);
    const int64_t t = n / g.m[2];
    iy = static_cast<int>(t % g.m[1]);
    ix = static_cast<int>(t / g.m[1]);
}

__device__ inline void node(int64_t n, const Grid64& g, int& jx, int& jy, int& jz) {
    jz = static_cast<int>(n % g.my[2]);
    const int64_t t = n / g.my[2];
    jy = static_cast<int>(t % g.my[1]);
    jx = static_cast<int>(t / g.my[1]);
}

// y_hat = P y at one voxel, then the clamped trilinear warp of T there and
// its derivative with respect to y_hat (slope 0 where a coordinate left the
// domain; the cell is clamped to [0, m-2] so the top edge is left-sided).
__global__ __launch_bounds__(kT) void k64_warp(Grid64 g, const double* __restrict__ y,
                                                const float* __restrict__ T,
                                                double* __restrict__ Ty,
                                                double* __restrict__ dT) {
    for (int64_t n = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x; n < g.n;
         n += static_cast<int64_t>(gridDim.x) * kT) {
        int i[3];
        voxel(n, g, i[0], i[1], i[2]);
        int j0[3];
        double w[3][2];
        for (int d = 0; d < 3; ++d) index_map(i[d], g.m[d], g.my[d], j0[d], w[d][0], w[d][1]);
        double yh[3];
        for (int c = 0; c < 3; ++c) {
            const double* yc = y + c * g.ny;
            double acc = 0.0;
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    for (int e = 0; e < 2; ++e) {
                        const int64_t k =
                            (static_cast<int64_t>(j0[0] + a) * g.my[1] + (j0[1] + b)) * g.my[2] +
                            (j0[2] + e);
                        acc += (w[0][a] * w[1][b]) * w[2][e] * yc[k];
                    }
            yh[c] = acc;
        }
        int i0[3];
        double f[3], s[3];
        for (int d = 0; d < 3; ++d) {
            double xi = yh[d] / g.h[d] - 0.5;
            const double top = static_cast<double>(g.m[d] - 1);
            s[d] = (xi >= 0.0 && xi <= top) ? 1.0 : 0.0;
            xi = fmin(fmax(xi, 0.0), top);
            i0[d] = min(static_cast<int>(floor(xi)), g.m[d] - 2);
            f[d] = xi - i0[d];
        }
        double ty = 0.0, dt[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 2; ++a) {
            const double wa = a ? f[0] : 1.0 - f[0], da = a ? 1.0 : -1.0;
            for (int b = 0; b < 2; ++b) {
                const double wb = b ? f[1] : 1.0 - f[1], db = b ? 1.0 : -1.0;
                for (int e = 0; e < 2; ++e) {
                    const double wc = e ? f[2] : 1.0 - f[2], dc = e ? 1.0 : -1.0;
                    const int64_t k =
                        (static_cast<int64_t>(i0[0] + a) * g.m[1] + (i0[1] + b)) * g.m[2] +
                        (i0[2] + e);
                    const double val = static_cast<double>(T[k]);
                    ty += wa * wb * wc * val;
                    dt[0] += da * wb * wc * val;
                    dt[1] += wa * db * wc * val;
                    dt[2] += wa * wb * dc * val;
                }
            }
        }
        Ty[n] = ty;
        for (int d = 0; d < 3; ++d) dT[d * g.n + n] = dt[d] * (s[d] / g.h[d]);
    }
}

// Central difference along axis d at voxel (i) with replicated ghost cells.
template <class V>
__device__ inline double cdiff(const V* u, const Grid64& g, const int i[3], int64_t n, int d) {
    const int64_t stride = d == 0 ? static_cast<int64_t>(g.m[1]) * g.m[2] : (d == 1 ? g.m[2] : 1);
    const int64_t up = i[d] < g.m[d] - 1 ? n + stride : n;
    const int64_t dn = i[d] > 0 ? n - stride : n;
    return (static_cast<double>(u[up]) - static_cast<double>(u[dn])) / (2.0 * g.h[d]);
}

// NGF terms of Eq. 2 at every voxel; v = dD/d(grad T_y) and per-workgroup
// partial sums of 1 - r^2.
__global__ __launch_bounds__(kT) void k64_ngf(Grid64 g, const double* __restrict__ Ty,
                                               const float* __restrict__ R, double tau,
                                               double rho, double hbar, double* __restrict__ v,
                                               double* __restrict__ dpart) {
    __shared__ double red[kT];
    double acc = 0.0;
    for (int64_t n = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x; n < g.n;
         n += static_cast<int64_t>(gridDim.x) * kT) {
        int i[3];
        voxel(n, g, i[0], i[1], i[2]);
        double gT[3], gR[3];
        for (int d = 0; d < 3; ++d) {
            gT[d] = cdiff(Ty, g, i, n, d);
            gR[d] = cdiff(R, g, i, n, d);
        }
        const double nT = sqrt(gT[0] * gT[0] + gT[1] * gT[1] + gT[2] * gT[2] + tau * tau);
        const double nR = sqrt(gR[0] * gR[0] + gR[1] * gR[1] + gR[2] * gR[2] + rho * rho);
        const double c = gT[0] * gR[0] + gT[1] * gR[1] + gT[2] * gR[2] + tau * rho;
        const double r = c / (nT * nR);
        acc += 1.0 - r * r;
        const double k = -hbar * r / (nT * nR);
        const double q = c / (nT * nT);
        for (int d = 0; d < 3; ++d) v[d * g.n + n] = k * (gR[d] - q * gT[d]);
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) dpart[blockIdx.x] = s;
}

// Adjoint of the clamped central difference along axis d at voxel i:
// (w[i-1] - w[i+1])/(2h) inside, -(w[0] + w[1])/(2h) at the first cell and
// (w[m-2] + w[m-1])/(2h) at the last (m >= 3).
__device__ inline double cdiff_adj(const double* w, const Grid64& g, const int i[3], int64_t n,
                                   int d) {
    const int64_t stride = d == 0 ? static_cast<int64_t>(g.m[1]) * g.m[2] : (d == 1 ? g.m[2] : 1);
    const double h2 = 2.0 * g.h[d];
    if (i[d] == 0) return -(w[n] + w[n + stride]) / h2;
    if (i[d] == g.m[d] - 1) return (w[n - stride] + w[n]) / h2;
    return (w[n - stride] - w[n + stride]) / h2;
}

// e = sum_d G_d^T v_d, then z_d = e dT_y/dy_hat_d in place of dT.
__global__ __launch_bounds__(kT) void k64_adjoint(Grid64 g, const double* __restrict__ v,
                                                   double* __restrict__ dTz) {
    for (int64_t n = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x; n < g.n;
         n += static_cast<int64_t>(gridDim.x) * kT) {
        int i[3];
        voxel(n, g, i[0], i[1], i[2]);
        double e = 0.0;
        for (int d = 0; d < 3; ++d) e += cdiff_adj(v + d * g.n, g, i, n, d);
        for (int d = 0; d < 3; ++d) dTz[d * g.n + n] = e * dTz[d * g.n + n];
    }
}

// Displacement u = y - X at node (j) of component c, X_d = j_d h^y_d.
__device__ inline double disp(const double* yc, const Grid64& g, const int j[3], int c) {
    const int64_t k = (static_cast<int64_t>(j[0]) * g.my[1] + j[1]) * g.my[2] + j[2];
    return yc[k] - j[c] * g.hy[c];
}

// Seven-point Laplacian with replicated ghost nodes of a node field given by
// a functor value(j).
template <class F>
__device__ inline double laplacian(const Grid64& g, const int j[3], F value) {
    const double u0 = value(j);
    double out = 0.0;
    for (int d = 0; d < 3; ++d) {
        int jp[3] = {j[0], j[1], j[2]}, jm[3] = {j[0], j[1], j[2]};
        jp[d] = min(j[d] + 1, g.my[d] - 1);
        jm[d] = max(j[d] - 1, 0);
        out += (value(jp) - 2.0 * u0 + value(jm)) / (g.hy[d] * g.hy[d]);
    }
    return out;
}

// A u for u = y - X, every component; per-workgroup partial sums of (A u)^2.
__global__ __launch_bounds__(kT) void k64_lap(Grid64 g, const double* __restrict__ y,
                                               double* __restrict__ Au,
                                               double* __restrict__ spart) {
    __shared__ double red[kT];
    double acc = 0.0;
    for (int64_t n = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x; n < g.ny;
         n += static_cast<int64_t>(gridDim.x) * kT) {
        int j[3];
        node(n, g, j[0], j[1], j[2]);
        for (int c = 0; c < 3; ++c) {
            const double* yc = y + c * g.ny;
            const double a = laplacian(g, j, [&](const int* q) { return disp(yc, g, q, c); });
            Au[c * g.ny + n] = a;
            acc += a * a;
        }
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) spart[blockIdx.x] = s;
}

// grad J at every node: P^T z (Eq. 3: the image points of the index sets
// Omega_x x Omega_y x Omega_z, each weighted by the product of its per-axis
// weights toward this node) plus alpha hbar^y A (A u).  Along an axis with
// ratio r = m / (m^y - 1), the points interpolated from node j are
// i = (j-1) r ... (j+1) r - 1, clipped to the grid.
__global__ __launch_bounds__(kT) void k64_node(Grid64 g, const double* __restrict__ z,
                                                const double* __restrict__ Au, double alpha,
                                                double hbary, double* __restrict__ grad) {
    for (int64_t n = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x; n < g.ny;
         n += static_cast<int64_t>(gridDim.x) * kT) {
        int j[3];
        node(n, g, j[0], j[1], j[2]);
        int lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
            const int r = g.m[d] / (g.my[d] - 1);
            lo[d] = max(0, (j[d] - 1) * r);
            hi[d] = min(g.m[d] - 1, (j[d] + 1) * r - 1);
        }
        double gd[3] = {0.0, 0.0, 0.0};
        for (int ix = lo[0]; ix <= hi[0]; ++ix) {
            int jx;
            double a0, a1;
            index_map(ix, g.m[0], g.my[0], jx, a0, a1);
            const double wx = jx == j[0] ? a0 : (jx + 1 == j[0] ? a1 : 0.0);
            for (int iy = lo[1]; iy <= hi[1]; ++iy) {
                int jy;
                double b0, b1;
                index_map(iy, g.m[1], g.my[1], jy, b0, b1);
                const double wy = jy == j[1] ? b0 : (jy + 1 == j[1] ? b1 : 0.0);
                for (int iz = lo[2]; iz <= hi[2]; ++iz) {
                    int jz;
                    double c0, c1;
                    index_map(iz, g.m[2], g.my[2], jz, c0, c1);
                    const double wz = jz == j[2] ? c0 : (jz + 1 == j[2] ? c1 : 0.0);
                    const double w = (wx * wy) * wz;
                    const int64_t k = (static_cast<int64_t>(ix) * g.m[1] + iy) * g.m[2] + iz;
                    for (int c = 0; c < 3; ++c) gd[c] += w * z[c * g.n + k];
                }
            }
        }
        for (int c = 0; c < 3; ++c) {
            const double* ac = Au + c * g.ny;
            const double gs = hbary * laplacian(g, j, [&](const int* q) {
                                  return ac[(static_cast<int64_t>(q[0]) * g.my[1] + q[1]) *
                                                g.my[2] +
                                            q[2]];
                              });
            grad[c * g.ny + n] = gd[c] + alpha * gs;
        }
    }
}

// D = (hbar/2) sum(1 - r^2), S = (hbar^y/2) sum (A u)^2, J = D + alpha S, from
// the kBlocks partial sums of each, in a fixed order.  out = {J, D, S}.
__global__ __launch_bounds__(kT) void k64_reduce(const double* __restrict__ dpart,
                                                  const double* __restrict__ spart,
                                                  double half_hbar, double half_hbary,
                                                  double alpha, double* __restrict__ out) {
    __shared__ double red[kT];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < kBlocks; k += kT) {
        a += dpart[k];
        b += spart[k];
    }
    const double sd = block_sum(a, red);
    __syncthreads();
    const double ss = block_sum(b, red);
    if (threadIdx.x == 0) {
        const double D = half_hbar * sd, S = half_hbary * ss;
        out[0] = D + alpha * S;
        out[1] = D;
        out[2] = S;
    }
}

}  // namespace

using namespace ngf_host;

#define F64CHK(ctx, expr)                                                              \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(ctx, NGF_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

extern "C" ngf_status ngf_eval_J_grad_f64(ngf_ctx* c, int32_t level, const double* y, double* J,
                                          double* grad, double* DS) {
    if (!c) return NGF_E_ARG;
    if (c->lv.empty()) return fail(c, NGF_E_STATE, "no pyramid");
    if (level < 0 || level >= static_cast<int>(c->lv.size()))
        return fail(c, NGF_E_LEVEL, "bad level");
    if (!y) return fail(c, NGF_E_ARG, "null y");
    const Level& L = c->lv[level];
    Grid64 g{};
    for (int d = 0; d < 3; ++d) {
        g.m[d] = L.m[d];
        g.my[d] = L.my[d];
        g.h[d] = L.h[d];
        g.hy[d] = L.hy[d];
    }
    g.n = L.N();
    g.ny = L.Ny();
    // scratch: T_y, dT (then z), v, A u, two sets of partial sums, {J, D, S}
    const size_t need = static_cast<size_t>(7 * g.n + 3 * g.ny + 2 * kBlocks + 3);
    if (need > c->f64_cap) {
        F64CHK(c, hipStreamSynchronize(c->stream));  // queued work may use the old buffer
        if (c->f64) (void)hipFree(c->f64);
        c->f64 = nullptr;
        c->f64_cap = 0;
        if ((c->faults & NGF_FAULT_ALLOC) ||
            hipMalloc(reinterpret_cast<void**>(&c->f64), need * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            c->f64 = nullptr;
            return fail(c, NGF_E_OOM, "hipMalloc of the float64 scratch failed");
        }
        c->f64_cap = need;
    }
    double* Ty = c->f64;
    double* dTz = Ty + g.n;
    double* v = dTz + 3 * g.n;
    double* Au = v + 3 * g.n;
    double* dpart = Au + 3 * g.ny;
    double* spart = dpart + kBlocks;
    double* out = spart + kBlocks;
    const double hbar = L.h[0] * L.h[1] * L.h[2];
    const double hbary = L.hy[0] * L.hy[1] * L.hy[2];
    hipStream_t s = c->stream;
    k64_warp<<<kBlocks, kT, 0, s>>>(g, y, L.T, Ty, dTz);
    k64_ngf<<<kBlocks, kT, 0, s>>>(g, Ty, L.R, c->p.tau, c->p.rho, hbar, v, dpart);
    k64_lap<<<kBlocks, kT, 0, s>>>(g, y, Au, spart);
    if (grad) {
        k64_adjoint<<<kBlocks, kT, 0, s>>>(g, v, dTz);
        k64_node<<<kBlocks, kT, 0, s>>>(g, dTz, Au, c->p.alpha, hbary, grad);
    }
    k64_reduce<<<1, kT, 0, s>>>(dpart, spart, 0.5 * hbar, 0.5 * hbary, c->p.alpha, out);
    F64CHK(c, hipGetLastError());
    if (J || DS) {
        double h3[3];
        F64CHK(c, hipMemcpyAsync(h3, out, sizeof(h3), hipMemcpyDeviceToHost, s));
        F64CHK(c, hipStreamSynchronize(s));
        if (J) *J = h3[0];
        if (DS) {
            DS[0] = h3[1];
            DS[1] = h3[2];
        }
        if (!std::isfinite(h3[0])) return fail(c, NGF_E_NONFINITE, "J is not finite");
    }
    return NGF_OK;
}
