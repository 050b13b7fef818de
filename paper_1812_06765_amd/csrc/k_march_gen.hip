// Image-grid pass for any deformation grid (per-axis node counts, grid
// ratios of 2 and more, integer or not), marching along x.  It computes what
// the other image passes compute -- P and the trilinear warp with float64
// coordinates (Sec. 2.1, Sec. 2.2 "Grid conversion"), the NGF term of Eq. 2
// with its matrix-free adjoint, and the tile-local part of the P^T gather of
// Eq. 3 -- but takes every grid-conversion index and weight from the exact
// integer index maps (image point i lies at node coordinate num/den with
// num = (2i+1)(n-1), den = 2m), so no ratio is built in.
//
// Organisation.  A workgroup of 512 threads owns a 32 x 32 (y, z) tile and a
// chunk of planes along x.  Thread t keeps the two tile voxels (t/32, t%32)
// and (t/32 + 16, t%32) for the whole march, plus (t < 272) one position of
// the two-voxel in-plane halo ring; the first 128 ring positions are the
// faces of the one-voxel halo, where the NGF adjoint needs v.  Step k warps
// plane p_w = x0 - 2 + k, evaluates the NGF term on plane p_w - 1 and the
// adjoint on plane p_w - 2.  Everything a step reads from LDS was written in
// an earlier step, so one barrier per step suffices:
//   * W writes T_y of p_w to one of two plane slots; V reads the other
//     (plane p_w - 1) for its in-plane differences.  Differences along x use
//     the thread's own warped values of planes p_w and p_w - 2 (registers).
//   * V keeps v_x in registers (the x adjoint needs only the thread's own
//     position) and writes v_y, v_z to double-buffered face-extended slots
//     that E reads one step later.
//   * E forms e = G^T v and dD/dy_hat = e dT_y/dy_hat in registers and adds
//     it, weighted along x, into per-voxel accumulators of the two node
//     planes the image plane touches.
//   * When a node plane is complete its accumulators go through LDS and are
//     reduced along z and y onto the tile's nodes, one stage per step
//     (write, z sums, y sums and store), in the slack of the following steps.
// The reference side of the NGF term (grad R and 1/(|grad R|^2 + rho^2)) is
// read from a per-level array prepared once per pyramid (k_rn).
#include "ngf_internal.h"

#include <math.h>

#include <atomic>

namespace ngf {

namespace {

constexpr int GT = 32;                  // in-plane tile extent (y and z)
constexpr int GH = GT + 4;              // two-voxel halo box extent
constexpr int GNH = GH * GH;            // 1296 warped positions per plane
constexpr int GNI = GT * GT;            // 1024 tile voxels per plane
constexpr int GRING = GNH - GNI;        // 272 halo positions
constexpr int GFACE = 4 * GT;           // 128 face positions of the one-voxel halo
constexpr int GNQ1 = 20;                // nodes per in-plane axis a halo box spans (ratio >= 2)
constexpr int GNQ = GNQ1 * GNQ1;
constexpr int GPMAX = GT / 2 + 2;       // nodes per tile and axis (ratio >= 2)
constexpr int GVY = (GT + 2) * GT;      // v_y slot: rows -1 .. 32, columns 0 .. 31
constexpr int GVZ = GT * (GT + 2);      // v_z slot: rows 0 .. 31, columns -1 .. 32

// LDS layout (bytes); doubles first for alignment
constexpr int L_Q = 0;                                   // 2 x 3 x GNQ doubles
constexpr int L_QW = L_Q + 2 * 3 * GNQ * 8;              // 2 x GH double2 (y, z)
constexpr int L_TY = L_QW + 2 * GH * 16;                 // 2 x GNH floats
constexpr int L_VY = L_TY + 2 * GNH * 4;                 // 2 x GVY floats
constexpr int L_VZ = L_VY + 2 * GVY * 4;                 // 2 x GVZ floats
constexpr int L_G = L_VZ + 2 * GVZ * 4;                  // 3 x GNI floats
constexpr int L_GZ = L_G + 3 * GNI * 4;                  // 3 x GT x GPMAX floats
constexpr int L_QJ = L_GZ + 3 * GT * GPMAX * 4;          // 2 x GH ints
constexpr int L_PW = L_QJ + 2 * GH * 4;                  // 2 x GT float2
constexpr int L_PJ = L_PW + 2 * GT * 8;                  // 2 x GT ints
constexpr int L_RG = L_PJ + 2 * GT * 4;                  // 2 x GPMAX int2 (voxel range per node)
constexpr int L_END = L_RG + 2 * GPMAX * 8;
static_assert(L_END <= 81920, "two workgroups per CU");

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, bytes, 0x00020000);
}
__device__ inline float bld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ inline float2 bld2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
}
__device__ inline float4 bld4(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]),
                       __uint_as_float(v[3]));
}

// Index map along one axis of m cells and n nodes (exact integers): node
// j0 and the float64 weights w0 = (den - r)/den, w1 = r/den (correctly
// rounded quotients).
struct Map1 {
    int j0;
    double w0, w1;
};
__device__ inline Map1 map1(int i, int m, int n) {
    const int num = (2 * i + 1) * (n - 1), den = 2 * m;
    Map1 r;
    r.j0 = num / den;
    const int rem = num - r.j0 * den;
    r.w1 = static_cast<double>(rem) / static_cast<double>(den);
    r.w0 = static_cast<double>(den - rem) / static_cast<double>(den);
    return r;
}
__device__ inline int map_j0(int i, int m, int n) { return ((2 * i + 1) * (n - 1)) / (2 * m); }

__device__ inline double wave_sum_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// halo-ring position s (< GRING) in the two-voxel box: the 128 faces of the
// one-voxel halo first (y faces, then z faces), then the outer ring and the
// corners of the one-voxel halo
__device__ inline void ring_pos(int s, int& by, int& bz) {
    if (s < 64) {
        by = s < 32 ? 1 : GT + 2;
        bz = 2 + (s & 31);
    } else if (s < 128) {
        const int q = s - 64;
        by = 2 + (q >> 1);
        bz = (q & 1) ? GT + 2 : 1;
    } else {
        const int o = s - 128;
        if (o < GH) {
            by = 0;
            bz = o;
        } else if (o < 2 * GH) {
            by = GH - 1;
            bz = o - GH;
        } else if (o < 2 * GH + 2 * (GT + 2)) {
            const int q = o - 2 * GH;
            by = 1 + (q >> 1);
            bz = (q & 1) ? GH - 1 : 0;
        } else {
            const int q = o - 2 * GH - 2 * (GT + 2);
            by = (q & 1) ? GT + 2 : 1;
            bz = (q & 2) ? GT + 2 : 1;
        }
    }
}

// KP tile voxels per thread: workgroups of 1024 / KP threads
template <int KP, bool GRAD, bool POW2>
__device__ __forceinline__ void gen_body(const ImagePassArgs& a, int CX, int block) {
    constexpr int GNT = GNI / KP;
    constexpr int NPOS = KP + 1;  // tile voxels, then the ring position
    constexpr int RK = KP;        // index of the ring position
    constexpr int GKQ = (3 * GNQ + GNT - 1) / GNT;
    static_assert(GNT >= GRING && GNT >= 128 + 2 * GT, "table and ring threads");
    extern __shared__ __align__(16) unsigned char gsm[];
    double* sQ = reinterpret_cast<double*>(gsm + L_Q);
    double2* sQW = reinterpret_cast<double2*>(gsm + L_QW);   // [axis][GH]
    float* sTy = reinterpret_cast<float*>(gsm + L_TY);
    float* sVy = reinterpret_cast<float*>(gsm + L_VY);
    float* sVz = reinterpret_cast<float*>(gsm + L_VZ);
    float* sG = reinterpret_cast<float*>(gsm + L_G);
    float* sGz = reinterpret_cast<float*>(gsm + L_GZ);
    int* sQJ = reinterpret_cast<int*>(gsm + L_QJ);          // [axis][GH]
    float2* sPW = reinterpret_cast<float2*>(gsm + L_PW);    // [axis][GT]
    int* sPJ = reinterpret_cast<int*>(gsm + L_PJ);          // [axis][GT]
    int2* sRG = reinterpret_cast<int2*>(gsm + L_RG);        // [axis][GPMAX]
    __shared__ double red[GNT / 64];

    const int t = threadIdx.x;
    const int tile = xcd_tile(block, a.ntx * a.nty * a.ntz);
    const int tz = tile % a.ntz;
    const int ty = (tile / a.ntz) % a.nty;
    const int tx = tile / (a.ntz * a.nty);
    const int x0 = tx * CX, y0 = ty * GT, z0 = tz * GT;
    const int mx = a.mx, my = a.my, mz = a.mz;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int sxT = my * mz;
    const int nnod = nx * ny * nz;
    const int xend = min(x0 + CX, mx);
    const int nstep = xend - x0 + 4;
    const int PX = a.px, PY = a.py, PZ = a.pz;
    // node bases: of the Q plane (halo box) and of the tile's P^T block
    const int qly = map_j0(max(y0 - 2, 0), my, ny), qlz = map_j0(max(z0 - 2, 0), mz, nz);
    const int nlox = map_j0(x0, mx, nx), nloy = map_j0(y0, my, ny), nloz = map_j0(z0, mz, nz);

    // ---- per-tile tables of the in-plane index maps ----------------------
    if (t < 2 * GH) {
        const int ax = t / GH, b = t - ax * GH;
        const int m = ax == 0 ? my : mz, n = ax == 0 ? ny : nz, o = ax == 0 ? y0 : z0;
        const Map1 mp = map1(clampi(o - 2 + b, 0, m - 1), m, n);
        sQJ[t] = mp.j0 - (ax == 0 ? qly : qlz);
        sQW[t] = make_double2(mp.w0, mp.w1);
    } else if (t >= 128 && t < 128 + 2 * GT) {
        const int q = t - 128, ax = q / GT, l = q - ax * GT;
        const int m = ax == 0 ? my : mz, n = ax == 0 ? ny : nz, o = ax == 0 ? y0 : z0;
        if (o + l < m) {
            const Map1 mp = map1(o + l, m, n);
            sPJ[q] = mp.j0 - (ax == 0 ? nloy : nloz);
            sPW[q] = make_float2(static_cast<float>(mp.w0), static_cast<float>(mp.w1));
        } else {
            sPJ[q] = -1000;  // outside the domain: in no node's range
            sPW[q] = make_float2(0.0f, 0.0f);
        }
    }
    __syncthreads();
    // voxel range of each of the tile's nodes (its index set restricted to
    // the tile): node n takes voxels with local node index n (weight w0) or
    // n - 1 (weight w1)
    if (t < 2 * GPMAX) {
        const int ax = t / GPMAX, n = t - ax * GPMAX;
        const int* pj = sPJ + ax * GT;
        int lo = GT, hi = -1;
        for (int l = 0; l < GT; ++l) {
            const int j = pj[l];
            if (j == n || j + 1 == n) {
                lo = min(lo, l);
                hi = max(hi, l);
            }
        }
        sRG[t] = make_int2(lo, hi);
    }

    // ---- buffers ---------------------------------------------------------
    const uint32_t plane4 = static_cast<uint32_t>(sxT) * 4u;
    const __amdgpu_buffer_rsrc_t rT = rsrc(a.T, static_cast<uint32_t>(mx) * plane4);
    const __amdgpu_buffer_rsrc_t rY = rsrc(a.y, 3u * static_cast<uint32_t>(nnod) * 4u);
    const uint32_t nplane4 = static_cast<uint32_t>(ny * nz) * 4u;

    // ---- the thread's positions ------------------------------------------
    // tile voxels kk < KP: (ly, lz) = ((t + kk GNT) / 32, t % 32); the ring
    // position kk = RK (t < GRING); box coordinates (by, bz), clamped global
    // (gy, gz)
    const bool ring = t < GRING;
    const bool face = t < GFACE;
    const bool fy = t < 64;  // a face position needs v_y (y face) or v_z (z face)
    const int lz0 = t & 31;
    int pby[NPOS], pbz[NPOS];
#pragma unroll
    for (int kk = 0; kk < KP; ++kk) {
        pby[kk] = ((t + kk * GNT) >> 5) + 2;
        pbz[kk] = lz0 + 2;
    }
    ring_pos(ring ? t : 0, pby[RK], pbz[RK]);
    auto gyof = [&](int kk) { return clampi(y0 - 2 + pby[kk], 0, my - 1); };
    auto gzof = [&](int kk) { return clampi(z0 - 2 + pbz[kk], 0, mz - 1); };
    // Q offset of each position (lower node pair), read from the tables below
    int qoff[NPOS];
    // Q plane entries of this thread: component, clamped in-plane node offset
    auto qld = [&](int k) -> uint32_t {
        const int i = min(t + k * GNT, 3 * GNQ - 1);
        const int c = i / GNQ, r = i - c * GNQ;
        const int gy = min(qly + r / GNQ1, ny - 1), gz = min(qlz + r % GNQ1, nz - 1);
        return static_cast<uint32_t>(c * nnod + gy * nz + gz) * 4u;
    };
    float qv0[GKQ], qv1[GKQ];
    double qwx0 = 1.0, qwx1 = 0.0;
    auto load_q = [&](int p) {
        const Map1 mp = map1(clampi(p, 0, mx - 1), mx, nx);
        qwx0 = mp.w0;
        qwx1 = mp.w1;
#pragma unroll
        for (int k = 0; k < GKQ; ++k) {
            const uint32_t o = qld(k);
            qv0[k] = bld(rY, o, static_cast<uint32_t>(mp.j0) * nplane4);
            qv1[k] = bld(rY, o, static_cast<uint32_t>(mp.j0 + 1) * nplane4);
        }
    };
    auto store_q = [&](int slot) {
        double* Q = sQ + slot * 3 * GNQ;
#pragma unroll
        for (int k = 0; k < GKQ; ++k) {
            const int i = t + k * GNT;
            if (i < 3 * GNQ)
                Q[i] = qwx0 * static_cast<double>(qv0[k]) + qwx1 * static_cast<double>(qv1[k]);
        }
    };
    __syncthreads();  // tables ready
#pragma unroll
    for (int kk = 0; kk < NPOS; ++kk) qoff[kk] = sQJ[pby[kk]] * GNQ1 + sQJ[GH + pbz[kk]];

    // ---- rolling state ----------------------------------------------------
    float tyv[NPOS][3];               // T_y of the positions at planes p_w - 2, p_w - 1, p_w
    float dT[3][KP][3];               // dT of planes p_w, p_w - 1, p_w - 2 (tile voxels)
    float vxs[2][KP];                 // v_x of planes p_v - 1, p_v - 2
    float accl[KP][3], acch[KP][3];   // P^T accumulators of node planes jA, jA + 1
#pragma unroll
    for (int kk = 0; kk < KP; ++kk) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            accl[kk][c] = acch[kk][c] = 0.0f;
            dT[0][kk][c] = dT[1][kk][c] = dT[2][kk][c] = 0.0f;
        }
        vxs[0][kk] = vxs[1][kk] = 0.0f;
    }
#pragma unroll
    for (int kk = 0; kk < NPOS; ++kk) tyv[kk][0] = tyv[kk][1] = tyv[kk][2] = 0.0f;
    int jA = nlox;
    int pendZ = -1, pendY = -1;      // node planes waiting for the z and y stages
    double dsum = 0.0;
    float* part = a.part + static_cast<int64_t>(tile) * 3 * PX * PY * PZ;
    const int NPB = PX * PY * PZ;

    // z stage of a completed node plane: sG -> sGz
    auto stage_z = [&]() {
        for (int i = t; i < 3 * GT * PZ; i += GNT) {
            const int n = i % PZ, row = i / PZ;  // row = (c, ly)
            const int2 rg = sRG[GPMAX + n];
            const float* g = sG + row * GT;
            float acc = 0.0f;
            for (int l = rg.x; l <= rg.y; ++l) {
                const float2 w = sPW[GT + l];
                acc = fmaf(sPJ[GT + l] == n ? w.x : w.y, g[l], acc);
            }
            sGz[i] = acc;
        }
    };
    // y stage: sGz -> the tile's P^T block at local node plane lx
    auto stage_y = [&](int lx) {
        for (int i = t; i < 3 * PY * PZ; i += GNT) {
            const int n = i % PZ, r = i / PZ;
            const int ny2 = r % PY, c = r / PY;
            const int2 rg = sRG[ny2];
            const float* g = sGz + c * GT * PZ + n;
            float acc = 0.0f;
            for (int l = rg.x; l <= rg.y; ++l) {
                const float2 w = sPW[l];
                acc = fmaf(sPJ[l] == ny2 ? w.x : w.y, g[l * PZ], acc);
            }
            part[c * NPB + lx * (PY * PZ) + ny2 * PZ + n] = acc;
        }
    };
    auto stage_w = [&](const float (&acc)[KP][3]) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int kk = 0; kk < KP; ++kk) sG[c * GNI + t + kk * GNT] = acc[kk][c];
    };

    load_q(x0 - 2);
    store_q(0);
    __syncthreads();

    for (int k = 0; k < nstep; ++k) {
        const int slot = k & 1;
        const int pw = x0 - 2 + k;
        // ------------- W: P and the warp of plane pw -----------------------
        {
            const double* Q = sQ + slot * 3 * GNQ;
            float tv[NPOS][8];
            float ff[NPOS][3], ss[KP][3];
            const double hh[3] = {a.hx, a.hy, a.hz};
            const double ih[3] = {a.ihx, a.ihy, a.ihz};
            const int mm[3] = {mx, my, mz};
#pragma unroll
            for (int kk = 0; kk < NPOS; ++kk) {
                if (kk == RK && !ring) continue;
                const double2 wy = sQW[pby[kk]], wz = sQW[GH + pbz[kk]];
                double yh[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double* q = Q + c * GNQ + qoff[kk];
                    const double c0 = wz.x * q[0] + wz.y * q[1];
                    const double c1 = wz.x * q[GNQ1] + wz.y * q[GNQ1 + 1];
                    yh[c] = wy.x * c0 + wy.y * c1;
                }
                int i0[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double xi = POW2 ? fma(yh[d], ih[d], -0.5) : yh[d] / hh[d] - 0.5;
                    const double xc = fmin(fmax(xi, 0.0), static_cast<double>(mm[d] - 1));
                    if (kk < KP) ss[kk < KP ? kk : 0][d] = xc == xi ? 1.0f : 0.0f;
                    const int i = min(static_cast<int>(xc), mm[d] - 2);
                    i0[d] = i;
                    ff[kk][d] = static_cast<float>(xc - static_cast<double>(i));
                }
                const uint32_t tb = static_cast<uint32_t>(i0[0] * sxT + i0[1] * mz + i0[2]) * 4u;
                const uint32_t row4 = static_cast<uint32_t>(mz) * 4u;
                const float2 t00 = bld2(rT, tb, 0u), t01 = bld2(rT, tb, row4);
                const float2 t10 = bld2(rT, tb, plane4), t11 = bld2(rT, tb, plane4 + row4);
                tv[kk][0] = t00.x;
                tv[kk][1] = t00.y;
                tv[kk][2] = t01.x;
                tv[kk][3] = t01.y;
                tv[kk][4] = t10.x;
                tv[kk][5] = t10.y;
                tv[kk][6] = t11.x;
                tv[kk][7] = t11.y;
            }
            // prefetch of the next Q plane's nodes (stored after V and E)
            if (k + 1 < nstep) load_q(pw + 1);
            float* Ty = sTy + slot * GNH;
#pragma unroll
            for (int kk = 0; kk < NPOS; ++kk) {
                if (kk == RK && !ring) continue;
                const float* v = tv[kk];
                const float fx = ff[kk][0], fyv = ff[kk][1], fz = ff[kk][2];
                const float qx = 1.0f - fx, qy = 1.0f - fyv, qz = 1.0f - fz;
                const float c00 = fmaf(fz, v[1], qz * v[0]), c01 = fmaf(fz, v[3], qz * v[2]);
                const float c10 = fmaf(fz, v[5], qz * v[4]), c11 = fmaf(fz, v[7], qz * v[6]);
                const float c0 = fmaf(fyv, c01, qy * c00), c1 = fmaf(fyv, c11, qy * c10);
                const float val = fmaf(fx, c1, qx * c0);
                Ty[pby[kk] * GH + pbz[kk]] = val;
                tyv[kk][0] = tyv[kk][1];
                tyv[kk][1] = tyv[kk][2];
                tyv[kk][2] = val;
                if (GRAD && kk < KP) {
                    const int q = kk < KP ? kk : 0;
                    const float d0 = c01 - c00, d1 = c11 - c10;
                    const float e00 = v[1] - v[0], e01 = v[3] - v[2], e10 = v[5] - v[4],
                                e11 = v[7] - v[6];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        dT[2][q][c] = dT[1][q][c];
                        dT[1][q][c] = dT[0][q][c];
                    }
                    dT[0][q][0] = (c1 - c0) * (ss[q][0] * a.fihx);
                    dT[0][q][1] = fmaf(fx, d1, qx * d0) * (ss[q][1] * a.fihy);
                    const float ez0 = fmaf(fyv, e01, qy * e00), ez1 = fmaf(fyv, e11, qy * e10);
                    dT[0][q][2] = fmaf(fx, ez1, qx * ez0) * (ss[q][2] * a.fihz);
                }
            }
        }
        // ------------- V: NGF on plane pv = pw - 1 -------------------------
        const int pv = pw - 1;
        float vxc[KP];
#pragma unroll
        for (int kk = 0; kk < KP; ++kk) vxc[kk] = 0.0f;
        if (pv >= max(x0 - 1, 0) && pv <= min(xend, mx - 1)) {
            const float* T0 = sTy + (slot ^ 1) * GNH;  // plane pv
            const bool dplane = pv >= x0 && pv < xend;
            const uint64_t rnb = static_cast<uint64_t>(pv) * static_cast<uint64_t>(sxT) * 16u;
            const __amdgpu_buffer_rsrc_t rR =
                rsrc(reinterpret_cast<const unsigned char*>(a.rn) + rnb,
                     static_cast<uint32_t>(sxT) * 16u);
            float* Vy = sVy + (pv & 1) * GVY;
            float* Vz = sVz + (pv & 1) * GVZ;
            const float tau = a.tau, rho = a.rho;
#pragma unroll
            for (int kk = 0; kk < NPOS; ++kk) {
                if (kk == RK && !face) continue;
                const int gy = gyof(kk), gz = gzof(kk);
                const int p = (gy - y0 + 2) * GH + (gz - z0 + 2);  // the clamped voxel
                const float4 rn = bld4(rR, static_cast<uint32_t>(gy * mz + gz) * 16u, 0u);
                const float gRx = rn.x, gRy = rn.y, gRz = rn.z, bb = rn.w;
                const float ibb = __builtin_amdgcn_rcpf(bb);
                const float gTx = (tyv[kk][2] - tyv[kk][0]) * a.i2hx;
                const float gTy = (T0[p + GH] - T0[p - GH]) * a.i2hy;
                const float gTz = (T0[p + 1] - T0[p - 1]) * a.i2hz;
                const float aa = fmaf(gTx, gTx, fmaf(gTy, gTy, fmaf(gTz, gTz, tau * tau)));
                const float ab = fmaf(gTx, gRx, fmaf(gTy, gRy, fmaf(gTz, gRz, tau * rho)));
                const float iaa = __builtin_amdgcn_rcpf(aa);
                // the position itself (unclamped): outside the domain its v is
                // the mirrored ghost of the adjoint stencil's end rows
                const int uy = y0 - 2 + pby[kk], uz = z0 - 2 + pbz[kk];
                if (kk < KP && dplane && uy < my && uz < mz) {
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
                    // v = -hbar ab/(aa^2 bb) (aa grad R - ab grad T), unfused
                    const float coef = -a.hbar * ab * (iaa * iaa) * ibb;
                    float wxx, wyy, wzz;
                    {
#pragma clang fp contract(off)
                        wxx = aa * gRx - ab * gTx;
                        wyy = aa * gRy - ab * gTy;
                        wzz = aa * gRz - ab * gTz;
                    }
                    const float vy = coef * wyy, vz = coef * wzz;
                    const float svy = uy != gy ? -vy : vy, svz = uz != gz ? -vz : vz;
                    if (kk < KP) {
                        vxc[kk < KP ? kk : 0] = coef * wxx;
                        const int ly = pby[kk] - 2;
                        Vy[(ly + 1) * GT + lz0] = svy;
                        Vz[ly * (GT + 2) + lz0 + 1] = svz;
                    } else if (fy) {
                        Vy[(pby[kk] - 1) * GT + (pbz[kk] - 2)] = svy;
                    } else {
                        Vz[(pby[kk] - 2) * (GT + 2) + (pbz[kk] - 1)] = svz;
                    }
                }
            }
        }
        // ------------- E: adjoint on plane pe = pw - 2, P^T along x --------
        const int pe = pw - 2;
        if (GRAD) {
            // pending reductions of completed node planes (one stage a step)
            if (pendY >= 0) {
                stage_y(pendY - nlox);
                pendY = -1;
            }
            if (pendZ >= 0) {
                stage_z();
                pendY = pendZ;
                pendZ = -1;
            }
            if (pe >= x0 && pe < xend) {
                const float* Vy = sVy + (pe & 1) * GVY;
                const float* Vz = sVz + (pe & 1) * GVZ;
                const Map1 mpx = map1(pe, mx, nx);
                if (mpx.j0 > jA) {  // node plane jA is complete
                    stage_w(accl);
                    pendZ = jA;
#pragma unroll
                    for (int kk = 0; kk < KP; ++kk)
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            accl[kk][c] = acch[kk][c];
                            acch[kk][c] = 0.0f;
                        }
                    jA += 1;
                }
                const float wx0 = static_cast<float>(mpx.w0), wx1 = static_cast<float>(mpx.w1);
#pragma unroll
                for (int kk = 0; kk < KP; ++kk) {
                    // v_x of planes pe - 1 and pe + 1; mirrored ghosts outside
                    const float vxm = pe > 0 ? vxs[1][kk] : -vxs[0][kk];
                    const float vxp = pe + 1 < mx ? vxc[kk] : -vxs[0][kk];
                    const float ex = vxm - vxp;
                    const int ly = pby[kk] - 2;
                    const float ey = Vy[ly * GT + lz0] - Vy[(ly + 2) * GT + lz0];
                    const float ez = Vz[ly * (GT + 2) + lz0] - Vz[ly * (GT + 2) + lz0 + 2];
                    const bool in = (y0 + ly < my) && (z0 + lz0 < mz);
                    const float e = in ? fmaf(ex, a.i2hx, fmaf(ey, a.i2hy, ez * a.i2hz)) : 0.0f;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const float g = e * dT[2][kk][c];
                        accl[kk][c] = fmaf(wx0, g, accl[kk][c]);
                        acch[kk][c] = fmaf(wx1, g, acch[kk][c]);
                    }
                }
            }
#pragma unroll
            for (int kk = 0; kk < KP; ++kk) {
                vxs[1][kk] = vxs[0][kk];
                vxs[0][kk] = vxc[kk];
            }
        }
        if (k + 1 < nstep) store_q(slot ^ 1);
        __syncthreads();
    }
    if (GRAD) {
        // drain: pending stages, then the last two node planes
        if (pendY >= 0) stage_y(pendY - nlox);
        __syncthreads();
        if (pendZ >= 0) {
            stage_z();
            __syncthreads();
            stage_y(pendZ - nlox);
            __syncthreads();
        }
        stage_w(accl);
        __syncthreads();
        stage_z();
        __syncthreads();
        stage_y(jA - nlox);
        stage_w(acch);
        __syncthreads();
        stage_z();
        __syncthreads();
        stage_y(jA + 1 - nlox);
    }
    // D partial of the tile: wave sums, then the waves in order
    double v = wave_sum_d(dsum);
    const int w = t >> 6;
    __syncthreads();
    if ((t & 63) == 0) red[w] = v;
    __syncthreads();
    if (t == 0) {
        double r = 0.0;
        for (int i = 0; i < GNT / 64; i += 2) r += red[i] + red[i + 1];
        a.dpart[tile] = r;
    }
}

template <int KP, bool GRAD, bool POW2>
__global__ __launch_bounds__(GNI / KP, 4) void k_image_gen(ImagePassArgs a, int CX) {
    if (a.gate && *a.gate == kOpNone) return;
    gen_body<KP, GRAD, POW2>(a, CX, blockIdx.x);
}

template <int KP, bool POW2>
__global__ __launch_bounds__(GNI / KP, 4) void k_image_gen_batch(const ImagePassArgs* args,
                                                                const BlockRef* blk) {
    const BlockRef e = blk[blockIdx.x];
    const int pair = __builtin_amdgcn_readfirstlane(e.pair);  // uniform: scalar loads
    if (pair < 0) return;
    const ImagePassArgs a = args[pair];
    if (a.gate && *a.gate == kOpNone) return;
    gen_body<KP, true, POW2>(a, __builtin_amdgcn_readfirstlane(a.cx),
                             __builtin_amdgcn_readfirstlane(e.block));
}

// Reference side of the NGF term per voxel: (grad R, |grad R|^2 + rho^2)
// by central differences with replicated ends -- the same expressions, in
// the same order, as the template side forms in the image passes, so that
// identical images give identical factors.
__global__ __launch_bounds__(kThreads) void k_rn(const float* __restrict__ R, float4* rn,
                                                 int mx, int my, int mz, float i2hx, float i2hy,
                                                 float i2hz, float rho) {
    const int64_t n = static_cast<int64_t>(mx) * my * mz;
    const int64_t sx = static_cast<int64_t>(my) * mz;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int z = static_cast<int>(i % mz);
        const int64_t q = i / mz;
        const int y = static_cast<int>(q % my);
        const int x = static_cast<int>(q / my);
        const float* p = R + i;
        const int64_t dxp = x < mx - 1 ? sx : 0, dxm = x > 0 ? sx : 0;
        const int dyp = y < my - 1 ? mz : 0, dym = y > 0 ? mz : 0;
        const int dzp = z < mz - 1 ? 1 : 0, dzm = z > 0 ? 1 : 0;
        const float gRx = (p[dxp] - p[-dxm]) * i2hx;
        const float gRy = (p[dyp] - p[-dym]) * i2hy;
        const float gRz = (p[dzp] - p[-dzm]) * i2hz;
        const float bb = fmaf(gRx, gRx, fmaf(gRy, gRy, fmaf(gRz, gRz, rho * rho)));
        rn[i] = make_float4(gRx, gRy, gRz, bb);
    }
}

constexpr int kGenKP = 1;  // tile voxels per thread of the general pass

template <bool POW2>
void launch_gen_t(const ImagePassArgs& a, int cx, hipStream_t s) {
    const int blocks = a.ntx * a.nty * a.ntz;
    if (a.want_grad)
        hipLaunchKernelGGL((k_image_gen<kGenKP, true, POW2>), dim3(blocks), dim3(GNI / kGenKP),
                           L_END, s, a, cx);
    else
        hipLaunchKernelGGL((k_image_gen<kGenKP, false, POW2>), dim3(blocks), dim3(GNI / kGenKP),
                           L_END, s, a, cx);
}

}  // namespace

void launch_image_gen(const ImagePassArgs& a, int cx, hipStream_t s) {
    if (a.pow2h)
        launch_gen_t<true>(a, cx, s);
    else
        launch_gen_t<false>(a, cx, s);
}

void launch_image_gen_batch(const ImagePassArgs* args, const BlockRef* blk, int nblk, bool pow2,
                            hipStream_t s) {
    if (nblk <= 0) return;
    if (pow2)
        hipLaunchKernelGGL((k_image_gen_batch<kGenKP, true>), dim3(nblk), dim3(GNI / kGenKP),
                           L_END, s, args, blk);
    else
        hipLaunchKernelGGL((k_image_gen_batch<kGenKP, false>), dim3(nblk), dim3(GNI / kGenKP),
                           L_END, s, args, blk);
}

void launch_rn(const float* R, float4* rn, int mx, int my, int mz, double hx, double hy,
               double hz, double rho, hipStream_t s) {
    const int64_t n = static_cast<int64_t>(mx) * my * mz;
    int64_t b = (n + kThreads - 1) / kThreads;
    if (b > 65536) b = 65536;
    hipLaunchKernelGGL(k_rn, dim3(static_cast<int>(b)), dim3(kThreads), 0, s, R, rn, mx, my, mz,
                       static_cast<float>(0.5 / hx), static_cast<float>(0.5 / hy),
                       static_cast<float>(0.5 / hz), static_cast<float>(rho));
}

int image_gen_slots() {
    static std::atomic<int> cache[16];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) dev = 0;
    std::atomic<int>& slot = cache[dev & 15];
    int v = slot.load();
    if (v > 0) return v;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_image_gen<kGenKP, true, true>,
                                                     GNI / kGenKP, L_END) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        cus = 256;
    (void)hipGetLastError();
    v = per_cu * cus;
    slot.store(v);
    return v;
}

}  // namespace ngf
