// Objective and gradient evaluation: J = D(R, T(P y)) + alpha S(y)
// (Sec. 2.1, Eq. 1), evaluated in the three steps of Sec. 2.2 ("Evaluating
// the objective function"): P, then the NGF distance of Eq. 2 with its
// matrix-free gradient, then P^T as a conflict-free gather (Eq. 3).
//
// Two kernels per evaluation, plus a one-block reduction:
//
// * image pass (one workgroup per image tile of kTX x kTY x kTZ voxels):
//     - stage the deformation nodes the tile needs in LDS;
//     - for the tile and a two-voxel halo: y_hat = P y (float64), the
//       trilinear warp T_y = T(y_hat) and, inside the tile, dT_y/dy_hat;
//     - for the tile and a one-voxel face halo: central differences of T_y
//       and R, the NGF term 1 - r^2 and v = dD/d(grad T_y);
//     - inside the tile: e = G^T v (adjoint stencil), dD/dy_hat = e dT_y/dy_hat;
//     - P^T restricted to the tile: separable weighted sums (z, y, x) onto the
//       (B+1)^3 nodes the tile touches, written as one partial block per tile.
//   Every write has one owner, so nothing races and nothing is atomic.
// * node pass (one workgroup per node tile): gathers the (at most 8) tile
//   partials of each node (this completes the sum of Eq. 3), adds
//   alpha grad S with grad S = hbar^y A(A(y - X)) from LDS halo tiles, and
//   writes grad J once.
// * reduce: fixed-order float64 sums of the block partials of D and S.
#include "ngf_internal.h"

#include <atomic>

#include <math.h>

namespace ngf {

namespace {

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ inline double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    return v;
}

// Sum over the workgroup (four wave64s) in a fixed order; result in thread 0.
__device__ inline double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    return r;
}
__device__ inline double block_max(double v, double* sh) {
    v = wave_max(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    return r;
}

// Continuous template index along one axis (float64), clamped, with the
// slope mask of the clamp, the cell and the float32 fraction.  The index is
// y_hat / h - 1/2 with a correctly rounded division: at the identity every
// index is an exact integer, and a product with a rounded 1/h can land one
// ulp below it and flip the cell (and so the one-sided derivative).
struct AxisCell {
    int i0;
    float f;
    float s;
};

template <bool POW2>
__device__ inline AxisCell axis_cell(double yhat, double h, double ih, int m) {
    // with a power-of-two spacing the reciprocal is exact and the product
    // rounds exactly like the quotient
    double xi = POW2 ? fma(yhat, ih, -0.5) : yhat / h - 0.5;
    const double hi = static_cast<double>(m - 1);
    const float s = (xi >= 0.0 && xi <= hi) ? 1.0f : 0.0f;
    xi = fmin(fmax(xi, 0.0), hi);
    const double fl = fmin(floor(xi), static_cast<double>(m - 2));
    AxisCell c;
    c.i0 = static_cast<int>(fl);
    c.f = static_cast<float>(xi - fl);
    c.s = s;
    return c;
}

template <int TX, int TY, int TZ, int RATIO>
struct ImageTile {
    static constexpr int H2X = TX + 4, H2Y = TY + 4, H2Z = TZ + 4;
    static constexpr int NH2 = H2X * H2Y * H2Z;
    static constexpr int H1X = TX + 2, H1Y = TY + 2, H1Z = TZ + 2;
    static constexpr int NH1 = H1X * H1Y * H1Z;
    static constexpr int NT = TX * TY * TZ;
    static constexpr int KT = NT / kThreads;
    static constexpr int BX = TX / RATIO, BY = TY / RATIO, BZ = TZ / RATIO;
    static constexpr int PX = BX + 1, PY = BY + 1, PZ = BZ + 1;
    static constexpr int NP = PX * PY * PZ;
    static constexpr int NBX = (TX + 4) / RATIO + 4, NBY = (TY + 4) / RATIO + 4,
                         NBZ = (TZ + 4) / RATIO + 4;
    static constexpr int NNODE = NBX * NBY * NBZ;
    static constexpr int VX = H1X * TY * TZ, VY = TX * H1Y * TZ, VZ = TX * TY * H1Z;
    static constexpr int NV = VX + VY + VZ;
    static constexpr int A = (NV > 3 * NNODE ? NV : 3 * NNODE);
    static constexpr int GZ = 3 * TX * TY * PZ, GY = 3 * TX * PY * PZ;
    static_assert(NT % kThreads == 0, "tile must be a multiple of the workgroup");
    static_assert(TX % RATIO == 0 && TY % RATIO == 0 && TZ % RATIO == 0, "ratio-aligned tile");
    static constexpr int B = (NH2 > 3 * NT ? NH2 : 3 * NT);
    static_assert(GZ + GY <= A, "P^T staging fits region A");
    static constexpr int LDS_FLOATS = A + B;
    static_assert(LDS_FLOATS * 4 <= 65536, "image tile fits 64 KiB of LDS");
};

// ATOMIC (differentiation form): instead of writing tile partials, stage 4
// adds each tile's P^T block into a.gy_atomic with float atomics, and stage 3
// scatters e W(i -> k) into a.gT_atomic (the transpose of the warp), both
// scaled by *a.gscale.
template <int TX, int TY, int TZ, int RATIO, bool GRAD, bool ATOMIC, bool POW2>
__device__ __forceinline__ void image_body(const ImagePassArgs& a, int block) {
    using L = ImageTile<TX, TY, TZ, RATIO>;
    extern __shared__ float smem[];
    float* sA = smem;                  // nodes, then v, then P^T staging
    float* sTy = smem + L::A;          // T_y on the two-voxel halo box
    float* sG = sTy;                   // dD/dy_hat on the tile (after v is formed)
    __shared__ double red[4];

    const int tile = xcd_tile(block, a.ntx * a.nty * a.ntz);
    const int tz = tile % a.ntz;
    const int ty = (tile / a.ntz) % a.nty;
    const int tx = tile / (a.ntz * a.nty);
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
    const int mx = a.mx, my = a.my, mz = a.mz;
    const int sxT = my * mz;

    // ---- stage 0: nodes of the two-voxel halo box into LDS --------------
    const int nlox = a.j0x[max(x0 - 2, 0)];
    const int nloy = a.j0y[max(y0 - 2, 0)];
    const int nloz = a.j0z[max(z0 - 2, 0)];
    const int nnod = a.nx * a.ny * a.nz;
    for (int i = threadIdx.x; i < 3 * L::NNODE; i += kThreads) {
        const int c = i / L::NNODE;
        const int r = i - c * L::NNODE;
        const int bz = r % L::NBZ;
        const int byy = (r / L::NBZ) % L::NBY;
        const int bx = r / (L::NBZ * L::NBY);
        const int gx = min(nlox + bx, a.nx - 1), gy = min(nloy + byy, a.ny - 1),
                  gz = min(nloz + bz, a.nz - 1);
        sA[i] = a.y[c * nnod + (gx * a.ny + gy) * a.nz + gz];
    }
    __syncthreads();

    // ---- stage 1: P and the warp ----------------------------------------
    // y_hat at image voxel (gx,gy,gz) (already clamped into the domain)
    auto warp_at = [&](int gx, int gy, int gz, float* dT, int* cb = nullptr,
                       float* cf = nullptr) -> float {
        const int jx = a.j0x[gx], jy = a.j0y[gy], jz = a.j0z[gz];
        const double ax1 = a.w1x[gx], ay1 = a.w1y[gy], az1 = a.w1z[gz];
        const double ax0 = a.w0x[gx], ay0 = a.w0y[gy], az0 = a.w0z[gz];
        const int base = ((jx - nlox) * L::NBY + (jy - nloy)) * L::NBZ + (jz - nloz);
        double yh[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float* Y = sA + c * L::NNODE + base;
            const double v000 = Y[0], v001 = Y[1];
            const double v010 = Y[L::NBZ], v011 = Y[L::NBZ + 1];
            const double v100 = Y[L::NBY * L::NBZ], v101 = Y[L::NBY * L::NBZ + 1];
            const double v110 = Y[L::NBY * L::NBZ + L::NBZ],
                         v111 = Y[L::NBY * L::NBZ + L::NBZ + 1];
            const double c00 = az0 * v000 + az1 * v001, c01 = az0 * v010 + az1 * v011;
            const double c10 = az0 * v100 + az1 * v101, c11 = az0 * v110 + az1 * v111;
            const double c0 = ay0 * c00 + ay1 * c01, c1 = ay0 * c10 + ay1 * c11;
            yh[c] = ax0 * c0 + ax1 * c1;
        }
        const AxisCell cx = axis_cell<POW2>(yh[0], a.hx, a.ihx, mx);
        const AxisCell cy = axis_cell<POW2>(yh[1], a.hy, a.ihy, my);
        const AxisCell cz = axis_cell<POW2>(yh[2], a.hz, a.ihz, mz);
        const float* Tb = a.T + cx.i0 * sxT + cy.i0 * mz + cz.i0;
        if (ATOMIC && cb != nullptr) {
            *cb = cx.i0 * sxT + cy.i0 * mz + cz.i0;
            cf[0] = cx.f;
            cf[1] = cy.f;
            cf[2] = cz.f;
        }
        const float v000 = Tb[0], v001 = Tb[1], v010 = Tb[mz], v011 = Tb[mz + 1];
        const float v100 = Tb[sxT], v101 = Tb[sxT + 1], v110 = Tb[sxT + mz],
                    v111 = Tb[sxT + mz + 1];
        // interpolation as (1-f) a + f b: exact at f = 0 and f = 1, so the
        // identity warp reproduces T bit for bit
        const float qx = 1.0f - cx.f, qy = 1.0f - cy.f, qz = 1.0f - cz.f;
        const float c00 = fmaf(cz.f, v001, qz * v000), c01 = fmaf(cz.f, v011, qz * v010);
        const float c10 = fmaf(cz.f, v101, qz * v100), c11 = fmaf(cz.f, v111, qz * v110);
        const float c0 = fmaf(cy.f, c01, qy * c00), c1 = fmaf(cy.f, c11, qy * c10);
        if (GRAD && dT != nullptr) {
            const float d0 = c01 - c00, d1 = c11 - c10;
            const float e00 = v001 - v000, e01 = v011 - v010, e10 = v101 - v100,
                        e11 = v111 - v110;
            dT[0] = (c1 - c0) * (cx.s * a.fihx);
            dT[1] = fmaf(cx.f, d1, qx * d0) * (cy.s * a.fihy);
            const float ez0 = fmaf(cy.f, e01, qy * e00), ez1 = fmaf(cy.f, e11, qy * e10);
            dT[2] = fmaf(cx.f, ez1, qx * ez0) * (cz.s * a.fihz);
        }
        return fmaf(cx.f, c1, qx * c0);
    };

    float dTk[L::KT][3];
    int cbk[ATOMIC ? L::KT : 1];
    float cfk[ATOMIC ? L::KT : 1][3];
#pragma unroll
    for (int k = 0; k < L::KT; ++k) {
        const int t = threadIdx.x + k * kThreads;
        const int lz = t % TZ, ly = (t / TZ) % TY, lx = t / (TZ * TY);
        const int gx = min(x0 + lx, mx - 1), gy = min(y0 + ly, my - 1), gz = min(z0 + lz, mz - 1);
        const float v = ATOMIC ? warp_at(gx, gy, gz, dTk[k], &cbk[ATOMIC ? k : 0],
                                         cfk[ATOMIC ? k : 0])
                               : warp_at(gx, gy, gz, dTk[k]);
        sTy[((lx + 2) * L::H2Y + (ly + 2)) * L::H2Z + (lz + 2)] = v;
    }
    // halo shell of the two-voxel box: x slabs, then y slabs, then z slabs
    {
        constexpr int S1 = 4 * L::H2Y * L::H2Z;
        constexpr int S2 = S1 + TX * 4 * L::H2Z;
        constexpr int S3 = S2 + TX * TY * 4;
        for (int s = threadIdx.x; s < S3; s += kThreads) {
            int bx, byy, bz;
            if (s < S1) {
                const int slab = s / (L::H2Y * L::H2Z);
                const int r = s - slab * (L::H2Y * L::H2Z);
                bx = slab < 2 ? slab : TX + slab;
                byy = r / L::H2Z;
                bz = r - byy * L::H2Z;
            } else if (s < S2) {
                const int q = s - S1;
                const int slab = (q / L::H2Z) & 3;
                bx = 2 + q / (4 * L::H2Z);
                byy = slab < 2 ? slab : TY + slab;
                bz = q % L::H2Z;
            } else {
                const int q = s - S2;
                const int slab = q & 3;
                const int r = q >> 2;
                bx = 2 + r / TY;
                byy = 2 + r % TY;
                bz = slab < 2 ? slab : TZ + slab;
            }
            const int gx = clampi(x0 - 2 + bx, 0, mx - 1), gy = clampi(y0 - 2 + byy, 0, my - 1),
                      gz = clampi(z0 - 2 + bz, 0, mz - 1);
            sTy[(bx * L::H2Y + byy) * L::H2Z + bz] = warp_at(gx, gy, gz, nullptr);
        }
    }
    __syncthreads();

    // ---- stage 2: NGF on the tile and its one-voxel face halo -------------
    float* sVx = sA;
    float* sVy = sA + L::VX;
    float* sVz = sA + L::VX + L::VY;
    double dsum = 0.0;
    const float tau = a.tau, rho = a.rho;
    for (int i = threadIdx.x; i < L::NH1; i += kThreads) {
        const int b1z = i % L::H1Z;
        const int b1y = (i / L::H1Z) % L::H1Y;
        const int b1x = i / (L::H1Z * L::H1Y);
        const int hx = (b1x == 0 || b1x == TX + 1), hy = (b1y == 0 || b1y == TY + 1),
                  hz = (b1z == 0 || b1z == TZ + 1);
        if (hx + hy + hz >= 2) continue;
        const int gx = x0 - 1 + b1x, gy = y0 - 1 + b1y, gz = z0 - 1 + b1z;
        const int cxp = clampi(gx, 0, mx - 1), cyp = clampi(gy, 0, my - 1),
                  czp = clampi(gz, 0, mz - 1);
        // position of the clamped voxel in the two-voxel box
        const int p = ((cxp - x0 + 2) * L::H2Y + (cyp - y0 + 2)) * L::H2Z + (czp - z0 + 2);
        constexpr int SX = L::H2Y * L::H2Z, SY = L::H2Z;
        const float gTx = (sTy[p + SX] - sTy[p - SX]) * a.i2hx;
        const float gTy = (sTy[p + SY] - sTy[p - SY]) * a.i2hy;
        const float gTz = (sTy[p + 1] - sTy[p - 1]) * a.i2hz;
        // reference differences straight from HBM/L2 (replicated ends)
        const float* Rp = a.R + cxp * sxT + cyp * mz + czp;
        const int dxp = (cxp < mx - 1) ? sxT : 0, dxm = (cxp > 0) ? sxT : 0;
        const int dyp = (cyp < my - 1) ? mz : 0, dym = (cyp > 0) ? mz : 0;
        const int dzp = (czp < mz - 1) ? 1 : 0, dzm = (czp > 0) ? 1 : 0;
        const float gRx = (Rp[dxp] - Rp[-dxm]) * a.i2hx;
        const float gRy = (Rp[dyp] - Rp[-dym]) * a.i2hy;
        const float gRz = (Rp[dzp] - Rp[-dzm]) * a.i2hz;
        const float aa = fmaf(gTx, gTx, fmaf(gTy, gTy, fmaf(gTz, gTz, tau * tau)));
        const float bb = fmaf(gRx, gRx, fmaf(gRy, gRy, fmaf(gRz, gRz, rho * rho)));
        const float ab = fmaf(gTx, gRx, fmaf(gTy, gRy, fmaf(gTz, gRz, tau * rho)));
        const float iaa = __builtin_amdgcn_rcpf(aa), ibb = __builtin_amdgcn_rcpf(bb);
        if (hx + hy + hz == 0 && gx < mx && gy < my && gz < mz) {
            // 1 - r^2 = (aa bb - ab^2) / (aa bb) with a = (grad T, tau), b = (grad R,
            // rho), products unfused: exactly 0 when a = b (aa = bb = ab bit for bit)
            float lag;
            {
#pragma clang fp contract(off)
                lag = aa * bb - ab * ab;
            }
            dsum += static_cast<double>(lag * iaa * ibb);
        }
        if (GRAD) {
            // v = -hbar r/(nT nR) (grad R - (c/nT^2) grad T)
            //   = -hbar ab/(aa^2 bb) (aa grad R - ab grad T),
            // with unfused products so that v is exactly 0 when grad T = grad R
            // (then ab = aa bit for bit and both products round alike)
            const float coef = -a.hbar * ab * (iaa * iaa) * ibb;
            float wx, wy, wz;
            {
#pragma clang fp contract(off)
                wx = aa * gRx - ab * gTx;
                wy = aa * gRy - ab * gTy;
                wz = aa * gRz - ab * gTz;
            }
            float vx = coef * wx;
            float vy = coef * wy;
            float vz = coef * wz;
            // outside the domain, the adjoint stencil's end rows are realised by a
            // mirrored ghost: v_d(m) = -v_d(m-1), v_d(-1) = -v_d(0)
            if (gx != cxp) vx = -vx;
            if (gy != cyp) vy = -vy;
            if (gz != czp) vz = -vz;
            if (!hy && !hz) sVx[(b1x * TY + (b1y - 1)) * TZ + (b1z - 1)] = vx;
            if (!hx && !hz) sVy[((b1x - 1) * L::H1Y + b1y) * TZ + (b1z - 1)] = vy;
            if (!hx && !hy) sVz[((b1x - 1) * TY + (b1y - 1)) * L::H1Z + b1z] = vz;
        }
    }
    const double dtot = block_sum(dsum, red);
    if (threadIdx.x == 0) a.dpart[tile] = dtot;
    if (!GRAD) return;
    const float gscale = (ATOMIC && a.gscale != nullptr) ? static_cast<float>(*a.gscale) : 1.0f;
    __syncthreads();

    // ---- stage 3: e = G^T v and dD/dy_hat on the tile ---------------------
#pragma unroll
    for (int k = 0; k < L::KT; ++k) {
        const int t = threadIdx.x + k * kThreads;
        const int lz = t % TZ, ly = (t / TZ) % TY, lx = t / (TZ * TY);
        const bool in = (x0 + lx < mx) && (y0 + ly < my) && (z0 + lz < mz);
        const float ex = sVx[(lx * TY + ly) * TZ + lz] - sVx[((lx + 2) * TY + ly) * TZ + lz];
        const float ey = sVy[(lx * L::H1Y + ly) * TZ + lz] - sVy[(lx * L::H1Y + ly + 2) * TZ + lz];
        const float ez = sVz[(lx * TY + ly) * L::H1Z + lz] - sVz[(lx * TY + ly) * L::H1Z + lz + 2];
        const float e = in ? fmaf(ex, a.i2hx, fmaf(ey, a.i2hy, ez * a.i2hz)) : 0.0f;
        sG[t] = e * dTk[k][0];
        sG[L::NT + t] = e * dTk[k][1];
        sG[2 * L::NT + t] = e * dTk[k][2];
        if (ATOMIC && a.gT_atomic != nullptr && in) {
            // dD/dT[k] += e W(i -> k) over the 8 corners of this voxel's cell
            const float es = e * gscale;
            const int b = cbk[ATOMIC ? k : 0];
            const float fx = cfk[ATOMIC ? k : 0][0], fy = cfk[ATOMIC ? k : 0][1],
                        fz = cfk[ATOMIC ? k : 0][2];
            const float qx = 1.0f - fx, qy = 1.0f - fy, qz = 1.0f - fz;
            float* G = a.gT_atomic + b;
            atomicAdd(G, es * qx * qy * qz);
            atomicAdd(G + 1, es * qx * qy * fz);
            atomicAdd(G + mz, es * qx * fy * qz);
            atomicAdd(G + mz + 1, es * qx * fy * fz);
            atomicAdd(G + sxT, es * fx * qy * qz);
            atomicAdd(G + sxT + 1, es * fx * qy * fz);
            atomicAdd(G + sxT + mz, es * fx * fy * qz);
            atomicAdd(G + sxT + mz + 1, es * fx * fy * fz);
        }
    }
    __syncthreads();
    if (ATOMIC && a.gy_atomic == nullptr) return;

    // ---- stage 4: P^T restricted to the tile (separable: z, y, x) ---------
    float* sGz = sA;             // [3][TX][TY][PZ]
    float* sGy = sA + L::GZ;     // [3][TX][PY][PZ]
    const int jz0 = z0 / RATIO, jy0 = y0 / RATIO, jx0 = x0 / RATIO;
    for (int i = threadIdx.x; i < L::GZ; i += kThreads) {
        const int nz = i % L::PZ;
        const int r = i / L::PZ;      // (c, lx, ly)
        const int jz = jz0 + nz;
        const int lo = max(0, RATIO * (nz - 1)), hi = min(TZ, RATIO * (nz + 1));
        const float* g = sG + r * TZ;  // sG[c][lx][ly][:]
        float acc = 0.0f;
        for (int lz = lo; lz < hi; ++lz) {
            const int iz = min(z0 + lz, mz - 1);
            const float w = (a.j0z[iz] == jz) ? a.w0z[iz] : a.w1z[iz];
            acc = fmaf(w, g[lz], acc);
        }
        sGz[i] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < L::GY; i += kThreads) {
        const int nz = i % L::PZ;
        const int ny = (i / L::PZ) % L::PY;
        const int r = i / (L::PZ * L::PY);  // (c, lx)
        const int jy = jy0 + ny;
        const int lo = max(0, RATIO * (ny - 1)), hi = min(TY, RATIO * (ny + 1));
        float acc = 0.0f;
        for (int ly = lo; ly < hi; ++ly) {
            const int iy = min(y0 + ly, my - 1);
            const float w = (a.j0y[iy] == jy) ? a.w0y[iy] : a.w1y[iy];
            acc = fmaf(w, sGz[(r * TY + ly) * L::PZ + nz], acc);
        }
        sGy[i] = acc;
    }
    __syncthreads();
    float* out = a.part + static_cast<int64_t>(tile) * 3 * L::NP;
    for (int i = threadIdx.x; i < 3 * L::NP; i += kThreads) {
        const int nz = i % L::PZ;
        const int ny = (i / L::PZ) % L::PY;
        const int nxl = (i / (L::PZ * L::PY)) % L::PX;
        const int c = i / L::NP;
        const int jx = jx0 + nxl;
        const int lo = max(0, RATIO * (nxl - 1)), hi = min(TX, RATIO * (nxl + 1));
        float acc = 0.0f;
        for (int lx = lo; lx < hi; ++lx) {
            const int ix = min(x0 + lx, mx - 1);
            const float w = (a.j0x[ix] == jx) ? a.w0x[ix] : a.w1x[ix];
            acc = fmaf(w, sGy[((c * TX + lx) * L::PY + ny) * L::PZ + nz], acc);
        }
        if (ATOMIC) {
            const int jy = jy0 + ny, jz = jz0 + nz;
            if (jx < a.nx && jy < a.ny && jz < a.nz)
                atomicAdd(a.gy_atomic + c * (a.nx * a.ny * a.nz) + (jx * a.ny + jy) * a.nz + jz,
                          acc * gscale);
        } else {
            out[i] = acc;
        }
    }
}

// ------------------------------------------------------------------------
// node pass
// ------------------------------------------------------------------------
template <int TX, int TY, int TZ, int RATIO, bool GRAD, bool ATOMIC, bool POW2>
__global__ __launch_bounds__(kThreads) void k_image_pass(ImagePassArgs a) {
    if (a.gate && *a.gate == kOpNone) return;
    image_body<TX, TY, TZ, RATIO, GRAD, ATOMIC, POW2>(a, blockIdx.x);
}

// Node pass, marching form: one workgroup per (component, NY x NZ node tile
// in (y, z), chunk of a.cxn node planes along x); thread t owns the in-plane node
// (t / NZ, t % NZ) of every plane of the chunk.  u = y - X is kept in three
// rolling LDS planes with a two-node in-plane halo, A u in three rolling
// planes with a one-node halo.  Ghost nodes replicate the boundary node
// (for u and for A u): in-plane through clamped loads and zero offsets, across
// planes by reading the boundary plane's slot.  Step k loads u of plane
// x0 - 2 + k, forms A u of plane x0 - 3 + k and A(A u) of plane x0 - 4 + k.
//
// The loop is kept free of per-lane branches and of per-plane index
// arithmetic on the scalar unit: the LDS planes are padded to whole passes of
// the workgroup (the surplus lanes work on a clamped copy and write into the
// padding), the plane slots rotate, the plane offsets advance by one plane
// per step, and lanes outside the grid compute on clamped data and store
// nothing.  GRAD: the gradient is wanted; GATHER: it collects the image-tile
// partials (else grad holds grad D on entry).
template <int NY, int NZ, bool GRAD, bool GATHER>
__device__ __forceinline__ void node_march_body(const NodePassArgs& a, int block) {
    static_assert(NY * NZ == kThreads, "one node per thread and plane");
    constexpr int UY = NY + 4, UZ = NZ + 4, NU = UY * UZ;  // u plane, halo 2
    constexpr int AY = NY + 2, AZ = NZ + 2, NA = AY * AZ;  // A u plane, halo 1
    constexpr int KU = (NU + kThreads - 1) / kThreads, KA = (NA + kThreads - 1) / kThreads;
    constexpr int SU = KU * kThreads, SA = KA * kThreads;  // padded plane sizes
    __shared__ float su[3 * SU];
    __shared__ float sAu[3 * SA];
    __shared__ double red[4];

    const int ntile = a.nbx * a.nby * a.nbz;
    const int bid = xcd_tile(block, 3 * ntile);
    const int c = bid / ntile;
    const int blk = bid - c * ntile;
    const int bz = blk % a.nbz;
    const int byy = (blk / a.nbz) % a.nby;
    const int bx = blk / (a.nbz * a.nby);
    const int x0 = bx * a.cxn, y0 = byy * NY, z0 = bz * NZ;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int nn = nx * ny * nz;
    const int plane = ny * nz;
    const int xend = min(x0 + a.cxn, nx);
    const int nstep = xend - x0 + 4;  // a chunk cut short by the grid stops after its last plane
    const int PX = a.px, PY = a.py, PZ = a.pz;
    const int NP = PX * PY * PZ;
    const float sc = (!GATHER && a.gscale != nullptr) ? static_cast<float>(*a.gscale) : 1.0f;
    const double hyc = c == 0 ? a.hyx : (c == 1 ? a.hyy : a.hyz);

    // this thread's node (y, z) and its fixed in-plane data
    const int ly = threadIdx.x / NZ, lz = threadIdx.x % NZ;
    const int gy = y0 + ly, gz = z0 + lz;
    const bool own = gy < ny && gz < nz;
    const int q = (ly + 1) * AZ + (lz + 1);
    const int dyp = gy + 1 < ny ? AZ : 0, dym = gy > 0 ? AZ : 0;
    const int dzp = gz + 1 < nz ? 1 : 0, dzm = gz > 0 ? 1 : 0;
    const int gofs = min(gy, ny - 1) * nz + min(gz, nz - 1);  // in-plane offset (clamped)
    // u halo entries of this thread (the padding lanes repeat the last one):
    // clamped in-plane offset and the coordinate X is taken along
    int uoff[KU];
    float ugc[KU];
#pragma unroll
    for (int k = 0; k < KU; ++k) {
        const int i = min(static_cast<int>(threadIdx.x) + k * kThreads, NU - 1);
        const int iy = i / UZ, iz = i - (i / UZ) * UZ;
        const int cy = clampi(y0 - 2 + iy, 0, ny - 1), cz = clampi(z0 - 2 + iz, 0, nz - 1);
        uoff[k] = cy * nz + cz;
        ugc[k] = static_cast<float>(c == 1 ? cy : cz);
    }
    // A u halo entries of this thread: their (clamped) node's place in the u plane
    int apos[KA];
#pragma unroll
    for (int k = 0; k < KA; ++k) {
        const int i = min(static_cast<int>(threadIdx.x) + k * kThreads, NA - 1);
        const int iy = i / AZ, iz = i - (i / AZ) * AZ;
        const int cy = clampi(y0 - 1 + iy, 0, ny - 1), cz = clampi(z0 - 1 + iz, 0, nz - 1);
        apos[k] = (cy - y0 + 2) * UZ + (cz - z0 + 2);
    }
    // gather of the image-tile partials (Eq. 3 completed): a node lies in the
    // blocks of at most two image tiles per axis, those of the first and the
    // last image point of its index set.  The (y, z) part of the node's place
    // in each (j = 2 oy + oz: second tile along y if oy, along z if oz) is
    // fixed over the chunk; the x part is the same for the whole workgroup
    // and is tabulated per plane of the chunk.  An entry that does not apply
    // reads offset 0 of the tile row and is not added.  The part array of one
    // x-slab of tiles is below 2^31 floats (checked by the host).
    int yzoff[4] = {0, 0, 0, 0};
    bool yzok[4] = {false, false, false, false};
    if constexpr (GATHER) {
        const NodeTiles ty = node_tiles(min(gy, ny - 1), a.my, ny, a.tey);
        const NodeTiles tz = node_tiles(min(gz, nz - 1), a.mz, nz, a.tez);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int oy = j >> 1, oz = j & 1;
            const int tty = oy ? ty.tb : ty.ta, ttz = oz ? tz.tb : tz.ta;
            const int lyy = oy ? ty.lb : ty.la, lzz = oz ? tz.lb : tz.la;
            yzok[j] = own && tty >= 0 && ttz >= 0;
            yzoff[j] = yzok[j] ? ((tty * a.ntz + ttz) * 3 + c) * NP + lyy * PZ + lzz : 0;
        }
    }
    const int64_t xslab = static_cast<int64_t>(a.nty) * a.ntz * 3 * NP;
    __shared__ int4 sxt[GATHER ? kNodeChunkMax : 1];
    for (int i = threadIdx.x; GATHER && i < xend - x0; i += kThreads) {
        const NodeTiles tx = node_tiles(x0 + i, a.mx, nx, a.tex);
        sxt[i] = make_int4(tx.ta, tx.la, tx.tb, tx.lb);
    }

    // y of this thread's entries of the u plane, loaded one step ahead so
    // that the loads overlap the previous plane's A u and output phases
    int64_t ycur = static_cast<int64_t>(c) * nn + static_cast<int64_t>(x0 - 2) * plane;
    float upre[KU];
    auto load_u = [&](int pu, int64_t yo) {
        if (pu < 0 || pu >= nx) return;  // planes outside the grid are never read
        const float* yp = a.y + yo;
#pragma unroll
        for (int kk = 0; kk < KU; ++kk) upre[kk] = yp[uoff[kk]];
    };
    load_u(x0 - 2, ycur);
    // this thread's output element: component c, plane po, in-plane offset
    int64_t grow = static_cast<int64_t>(c) * nn + static_cast<int64_t>(x0) * plane + gofs;
    // slots of the three rolling planes: s0 = k mod 3, s1 = (k + 1) mod 3, s2 = (k + 2) mod 3
    int s0 = 0, s1 = 1, s2 = 2;
    double ssum = 0.0, gmax = 0.0, g2 = 0.0;
    for (int k = 0; k < nstep; ++k) {
        // u of plane pu
        const int pu = x0 - 2 + k;
        if (pu >= 0 && pu < nx) {
            float* U = su + s0 * SU;
            const double gx = static_cast<double>(pu);
#pragma unroll
            for (int kk = 0; kk < KU; ++kk) {
                const double gcd = c == 0 ? gx : static_cast<double>(ugc[kk]);
                U[threadIdx.x + kk * kThreads] =
                    static_cast<float>(static_cast<double>(upre[kk]) - gcd * hyc);
            }
        }
        ycur += plane;
        if (k + 1 < nstep) load_u(pu + 1, ycur);
        __syncthreads();
        // A u of plane pa, from u planes pa - 1, pa, pa + 1 (replicated ghosts)
        const int pa = pu - 1;
        if (pa >= 0 && pa < nx) {
            const float* U0 = su + s2 * SU;                        // plane pa
            const float* Um = pa > 0 ? su + s1 * SU : U0;          // plane pa - 1
            const float* Up = pa + 1 < nx ? su + s0 * SU : U0;     // plane pa + 1
            float* A = sAu + s0 * SA;
#pragma unroll
            for (int kk = 0; kk < KA; ++kk) {
                const int p = apos[kk];
                const float u0 = U0[p];
                const float lx = Up[p] - 2.0f * u0 + Um[p];
                const float lyv = U0[p + UZ] - 2.0f * u0 + U0[p - UZ];
                const float lzv = U0[p + 1] - 2.0f * u0 + U0[p - 1];
                A[threadIdx.x + kk * kThreads] = fmaf(lx, a.ihy2x, fmaf(lyv, a.ihy2y, lzv * a.ihy2z));
            }
        }
        __syncthreads();
        // A(A u) and the gradient at plane po
        const int po = pu - 2;
        if (po >= x0 && po < xend) {
            const float* A0 = sAu + s2 * SA;                       // plane po
            const float* Am = po > 0 ? sAu + s1 * SA : A0;         // plane po - 1
            const float* Ap = po + 1 < nx ? sAu + s0 * SA : A0;    // plane po + 1
            const float au = A0[q];
            ssum += own ? static_cast<double>(au) * static_cast<double>(au) : 0.0;
            if (GRAD) {
                float gd = 0.0f;
                if (!GATHER) {
                    gd = a.grad[grow];
                } else {
                    // Eq. 3 completed: the (at most 8) image-tile partials of the
                    // node, in the order (ox, oy, oz)
                    const int4 xt = sxt[po - x0];
#pragma unroll
                    for (int ox = 0; ox < 2; ++ox) {
                        const int ttx = ox ? xt.z : xt.x;
                        if (ttx < 0) continue;
                        const float* px = a.part + ttx * xslab + (ox ? xt.w : xt.y) * (PY * PZ);
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const float v = px[yzoff[j]];
                            gd = yzok[j] ? gd + v : gd;
                        }
                    }
                }
                const float lxx = Ap[q] - 2.0f * au + Am[q];
                const float lyy = A0[q + dyp] - 2.0f * au + A0[q - dym];
                const float lzz = A0[q + dzp] - 2.0f * au + A0[q - dzm];
                const float aau = fmaf(lxx, a.ihy2x, fmaf(lyy, a.ihy2y, lzz * a.ihy2z));
                const float g = fmaf(a.alpha_hbary * sc, aau, gd);
                if (own) a.grad[grow] = g;
                gmax = own ? fmax(gmax, static_cast<double>(fabsf(g))) : gmax;
                g2 += own ? static_cast<double>(g) * static_cast<double>(g) : 0.0;
                grow += plane;
            }
        }
        const int t = s0;
        s0 = s1;
        s1 = s2;
        s2 = t;
    }
    const double st = block_sum(ssum, red);
    if (threadIdx.x == 0) a.spart[bid] = st;
    if (GRAD) {
        const double gm = block_max(gmax, red);
        const double gq = block_sum(g2, red);
        if (threadIdx.x == 0) {
            a.gpart[2 * bid] = gm;
            a.gpart[2 * bid + 1] = gq;
        }
    }
}

// GRAD: the gradient is wanted; GATHER: it collects the image-tile partials
template <bool GRAD, bool GATHER>
__global__ __launch_bounds__(kThreads) void k_node_pass(NodePassArgs a) {
    if (a.gate && *a.gate == kOpNone) return;
    node_march_body<kNMY, kNMZ, GRAD, GATHER>(a, blockIdx.x);
}

// the batched rounds always want the gradient gathered from the image pass
__global__ __launch_bounds__(kThreads) void k_node_pass_batch(const NodePassArgs* args,
                                                              const BlockRef* blk) {
    const BlockRef e = blk[blockIdx.x];
    if (e.pair < 0) return;
    const NodePassArgs& a = args[e.pair];
    if (a.gate && *a.gate == kOpNone) return;
    node_march_body<kNMY, kNMZ, true, true>(a, e.block);
}

template <int TX, int TY, int TZ, int RATIO, bool POW2>
__global__ __launch_bounds__(kThreads) void k_image_pass_batch(const ImagePassArgs* args,
                                                               const BlockRef* blk) {
    const BlockRef e = blk[blockIdx.x];
    if (e.pair < 0) return;
    const ImagePassArgs& a = args[e.pair];
    if (a.gate && *a.gate == kOpNone) return;
    image_body<TX, TY, TZ, RATIO, true, false, POW2>(a, e.block);
}

template <int TX, int TY, int TZ, int RATIO>
void launch_image_tile(const ImagePassArgs& a, hipStream_t s) {
    using L = ImageTile<TX, TY, TZ, RATIO>;
    const int blocks = a.ntx * a.nty * a.ntz;
    const size_t lds = sizeof(float) * L::LDS_FLOATS;
    if (a.want_grad) {
        if (a.pow2h)
            hipLaunchKernelGGL((k_image_pass<TX, TY, TZ, RATIO, true, false, true>),
                               dim3(blocks), dim3(kThreads), lds, s, a);
        else
            hipLaunchKernelGGL((k_image_pass<TX, TY, TZ, RATIO, true, false, false>),
                               dim3(blocks), dim3(kThreads), lds, s, a);
    } else {
        if (a.pow2h)
            hipLaunchKernelGGL((k_image_pass<TX, TY, TZ, RATIO, false, false, true>),
                               dim3(blocks), dim3(kThreads), lds, s, a);
        else
            hipLaunchKernelGGL((k_image_pass<TX, TY, TZ, RATIO, false, false, false>),
                               dim3(blocks), dim3(kThreads), lds, s, a);
    }
}

template <int TX, int TY, int TZ, int RATIO>
void launch_image_tile_atomic(const ImagePassArgs& a, hipStream_t s) {
    using L = ImageTile<TX, TY, TZ, RATIO>;
    const int blocks = a.ntx * a.nty * a.ntz;
    const size_t lds = sizeof(float) * L::LDS_FLOATS;
    if (a.pow2h)
        hipLaunchKernelGGL((k_image_pass<TX, TY, TZ, RATIO, true, true, true>), dim3(blocks),
                           dim3(kThreads), lds, s, a);
    else
        hipLaunchKernelGGL((k_image_pass<TX, TY, TZ, RATIO, true, true, false>), dim3(blocks),
                           dim3(kThreads), lds, s, a);
}

template <int RATIO>
void launch_image_ratio_atomic(const ImagePassArgs& a, int variant, hipStream_t s) {
    if (variant == kTile3DTiny)
        launch_image_tile_atomic<4, 4, 16, RATIO>(a, s);
    else if (variant == kTile3DSmall)
        launch_image_tile_atomic<4, 8, 32, RATIO>(a, s);
    else
        launch_image_tile_atomic<kTX, kTY, kTZ, RATIO>(a, s);
}

template <int TX, int TY, int TZ, int RATIO>
void launch_image_tile_batch(const ImagePassArgs* args, const BlockRef* blk, int nblk, bool pow2,
                             hipStream_t s) {
    using L = ImageTile<TX, TY, TZ, RATIO>;
    const size_t lds = sizeof(float) * L::LDS_FLOATS;
    if (pow2)
        hipLaunchKernelGGL((k_image_pass_batch<TX, TY, TZ, RATIO, true>), dim3(nblk),
                           dim3(kThreads), lds, s, args, blk);
    else
        hipLaunchKernelGGL((k_image_pass_batch<TX, TY, TZ, RATIO, false>), dim3(nblk),
                           dim3(kThreads), lds, s, args, blk);
}

template <int RATIO>
void launch_image_ratio_batch(const ImagePassArgs* args, const BlockRef* blk, int nblk,
                              int variant, bool pow2, hipStream_t s) {
    if (variant == kTile3DSmall)
        launch_image_tile_batch<4, 8, 32, RATIO>(args, blk, nblk, pow2, s);
    else if (variant == kTile3DTiny)
        launch_image_tile_batch<4, 4, 16, RATIO>(args, blk, nblk, pow2, s);
    else
        launch_image_tile_batch<kTX, kTY, kTZ, RATIO>(args, blk, nblk, pow2, s);
}

template <int RATIO>
void launch_image_ratio(const ImagePassArgs& a, int variant, hipStream_t s) {
    if (variant == kTile3DSmall)
        launch_image_tile<4, 8, 32, RATIO>(a, s);
    else if (variant == kTile3DTiny)
        launch_image_tile<4, 4, 16, RATIO>(a, s);
    else
        launch_image_tile<kTX, kTY, kTZ, RATIO>(a, s);
}

}  // namespace

// 3D-tile variants (kTile3D, kTile3DSmall, kTile3DTiny)
void launch_image_pass(const ImagePassArgs& a, int ratio, int variant, hipStream_t s) {
    if (ratio == 2)
        launch_image_ratio<2>(a, variant, s);
    else if (ratio == 4)
        launch_image_ratio<4>(a, variant, s);
}

// gradient form only (the batched rounds always want the gradient)
void launch_image_pass_batch(const ImagePassArgs* args, const BlockRef* blk, int nblk, int ratio,
                             int variant, bool pow2, hipStream_t s) {
    if (nblk <= 0) return;
    if (ratio == 2)
        launch_image_ratio_batch<2>(args, blk, nblk, variant, pow2, s);
    else if (ratio == 4)
        launch_image_ratio_batch<4>(args, blk, nblk, variant, pow2, s);
}

void launch_node_pass_batch(const NodePassArgs* args, const BlockRef* blk, int nblk,
                            hipStream_t s) {
    if (nblk <= 0) return;
    hipLaunchKernelGGL(k_node_pass_batch, dim3(nblk), dim3(kThreads), 0, s, args, blk);
}

void launch_image_pass_atomic(const ImagePassArgs& a, int ratio, int variant, hipStream_t s) {
    if (ratio == 2)
        launch_image_ratio_atomic<2>(a, variant, s);
    else if (ratio == 4)
        launch_image_ratio_atomic<4>(a, variant, s);
}

int node_march_slots() {
    static std::atomic<int> cache[16];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) dev = 0;
    std::atomic<int>& slot = cache[dev & 15];
    int v = slot.load();
    if (v > 0) return v;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_node_pass<true, true>, kThreads,
                                                     0) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 8;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        cus = 256;
    (void)hipGetLastError();
    v = per_cu * cus;
    slot.store(v);
    return v;
}

void launch_node_pass(const NodePassArgs& a, hipStream_t s) {
    const int blocks = 3 * a.nbx * a.nby * a.nbz;
    if (!a.want_grad)
        hipLaunchKernelGGL((k_node_pass<false, false>), dim3(blocks), dim3(kThreads), 0, s, a);
    else if (a.gather)
        hipLaunchKernelGGL((k_node_pass<true, true>), dim3(blocks), dim3(kThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_node_pass<true, false>), dim3(blocks), dim3(kThreads), 0, s, a);
}

}  // namespace ngf
