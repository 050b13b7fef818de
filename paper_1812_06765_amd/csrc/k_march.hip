// Image-grid pass, marching form.  Same arithmetic as k_image_pass (P and the
// warp with float64 coordinates, NGF term of Eq. 2, its adjoint stencil, the
// tile-local part of the P^T gather of Eq. 3), organised for fewer redundant
// voxels: a workgroup owns a (y, z) tile of TY x TZ voxels and a chunk of CX
// planes along x (the slowest axis) and walks the planes in order, keeping
// rolling planes in LDS.  Halos then exist only inside a plane (two voxels
// for the warped template, one for v) plus four planes per chunk, instead of
// in all three directions.
//
// Per step k (plane p_w = x0 - 2 + k enters):
//   W  warp plane p_w (tile + in-plane halo 2); stage R of plane p_w - 1
//   V  NGF on plane p_v = p_w - 1 (tile + in-plane face halo 1): D term, v
//   E  adjoint on plane p_e = p_w - 2 (tile): e = G^T v, dD/dy_hat = e dT
//   Z  P^T along z of plane p_e
//   Y  P^T along y, then along x into two register accumulators (the two
//      node planes the image plane touches); build the x-interpolated node
//      plane used by the next W
// Ghost planes of the x adjoint stencil (x = -1, x = m_x) are not computed:
// E substitutes v_x(-1) = -v_x(0) and v_x(m_x) = -v_x(m_x - 1) directly.
//
// The P^T partial sums are written in the tile layout the node pass reads:
// tile (chunk, ty, tz) owns node block [x0/R, x0/R + CX/R] x [...] x [...].
#include "ngf_internal.h"

#include <math.h>

#include <atomic>
#include <type_traits>

namespace ngf {

namespace {

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Raw buffer access to R, T and y: byte offsets in 32 bits (the host keeps
// the images below 2^30 voxels), the uniform part of an offset in a scalar
// register, no 64-bit address arithmetic per load.  A load past the buffer
// size returns 0 instead of faulting.
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const float* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), 0, bytes, 0x00020000);
}
__device__ inline float bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ inline float2 bload2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
}

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// threads of the marching workgroup: 256 (512 for the 32 x 32 tile, so that
// every thread keeps two voxels of a plane)
template <int TY, int TZ>
constexpr int march_threads() {
    return TY == 32 && TZ == 32 ? 512 : kThreads;
}

template <int TY, int TZ, int R>
struct March {
    static constexpr int NT = march_threads<TY, TZ>();
    static constexpr int H2Y = TY + 4, H2Z = TZ + 4, NH2 = H2Y * H2Z;
    static constexpr int H1Y = TY + 2, H1Z = TZ + 2;
    static constexpr int NI = TY * TZ, KP = NI / NT;
    static constexpr int NRING2 = NH2 - NI;             // in-plane halo-2 ring
    static constexpr int NRING1 = 2 * TZ + 2 * TY;      // in-plane face halo-1 ring
    static constexpr int BY = TY / R, BZ = TZ / R, PY = BY + 1, PZ = BZ + 1;
    static constexpr int NOUT = 3 * PY * PZ, KO = (NOUT + NT - 1) / NT;
    static constexpr int NQY = TY / R + 4, NQZ = TZ / R + 4, NQ = NQY * NQZ;
    static constexpr int GZ = 3 * TY * PZ;
    // LDS layout (floats)
    static constexpr int OFF_TY = 0;                          // 3 x NH2
    static constexpr int OFF_R = OFF_TY + 3 * NH2;            // NH2
    static constexpr int OFF_VX = OFF_R + NH2;                // 3 x NI
    static constexpr int OFF_VY = OFF_VX + 3 * NI;            // 2 x H1Y x TZ
    static constexpr int OFF_VZ = OFF_VY + 2 * H1Y * TZ;      // 2 x TY x H1Z
    static constexpr int OFF_G = OFF_VZ + 2 * TY * H1Z;       // max(3 NI, 2 x 3 NQ): sG or Q
    static constexpr int SZ_G = (3 * NI > 6 * NQ ? 3 * NI : 6 * NQ);
    static constexpr int OFF_GZ = OFF_G + SZ_G;               // GZ
    static constexpr int LDS_FLOATS = OFF_GZ + GZ;
    static_assert(NI % NT == 0, "tile plane must be a multiple of the workgroup");
    static_assert(TY % R == 0 && TZ % R == 0, "ratio-aligned tile");
    static_assert((OFF_G % 2) == 0, "double alignment of Q");
    static_assert(NRING1 <= NT, "face ring in one pass");
    static_assert(LDS_FLOATS * 4 <= 81920, "two workgroups per CU");
};

// image index -> node index and the two weights along one axis, for a
// power-of-two ratio: voxel i = q R + k lies at node coordinate q + (2k+1)/(2R)
template <int R>
__device__ inline int node_of(int i) {
    return i / R;
}
template <int R>
__device__ inline float w1_of(int i) {
    return static_cast<float>(2 * (i % R) + 1) * (0.5f / R);
}

// position of face-halo ring entry s (< 2 TZ + 2 TY) in the one-voxel halo box
template <int TY, int TZ>
__device__ inline void ring1_pos_t(int s, int& b1y, int& b1z) {
    if (s < 2 * TZ) {
        b1y = s < TZ ? 0 : TY + 1;
        b1z = 1 + (s % TZ);
    } else {
        const int q = s - 2 * TZ;
        b1y = 1 + (q >> 1);
        b1z = (q & 1) ? TZ + 1 : 0;
    }
}

template <int TY, int TZ, int R, bool GRAD, bool POW2>
__device__ __forceinline__ void march_body(const ImagePassArgs& a, int CX, int block) {
    using L = March<TY, TZ, R>;
    constexpr int NT = L::NT;
    auto ring1_pos = [](int s, int& b1y, int& b1z) { ring1_pos_t<TY, TZ>(s, b1y, b1z); };
    extern __shared__ float smem[];
    float* sTy = smem + L::OFF_TY;
    float* sR = smem + L::OFF_R;
    float* sVx = smem + L::OFF_VX;
    float* sVy = smem + L::OFF_VY;
    float* sVz = smem + L::OFF_VZ;
    float* sG = smem + L::OFF_G;
    double* sQ = reinterpret_cast<double*>(smem + L::OFF_G);
    float* sGz = smem + L::OFF_GZ;
    __shared__ double red[NT / 64];

    // tile decode, spread over the XCDs so that neighbouring tiles share an L2
    const int tile = xcd_tile(block, a.ntx * a.nty * a.ntz);
    const int tz = tile % a.ntz;
    const int ty = (tile / a.ntz) % a.nty;
    const int tx = tile / (a.ntz * a.nty);
    const int x0 = tx * CX, y0 = ty * TY, z0 = tz * TZ;
    const int mx = a.mx, my = a.my, mz = a.mz;
    const int sxT = my * mz;
    const int nnod = a.nx * a.ny * a.nz;
    const int qly = max(y0 - 2, 0) / R, qlz = max(z0 - 2, 0) / R;
    const int jx_first = x0 / R;
    const int xend = min(x0 + CX, mx);  // first plane past the chunk (in the domain)
    const uint32_t nbytes = static_cast<uint32_t>(mx) * static_cast<uint32_t>(sxT) * 4u;
    const __amdgpu_buffer_rsrc_t rT = make_rsrc(a.T, nbytes), rR = make_rsrc(a.R, nbytes);
    const __amdgpu_buffer_rsrc_t rY = make_rsrc(a.y, 3u * static_cast<uint32_t>(nnod) * 4u);
    const uint32_t plane4 = static_cast<uint32_t>(sxT) * 4u;  // bytes per image plane
    // steps: the chunk's planes plus two lead-in and two lead-out planes; a
    // chunk cut short by the domain stops after its last plane
    const int nstep = xend - x0 + 4;

    // x-interpolated node plane for image plane p (clamped), float64, into sQ.
    // The node values are loaded into registers one phase ahead of the store
    // (load_q during the warp phase, store_q after the last read of sG), so
    // their latency overlaps the warp's gathers.
    constexpr int KQ = (3 * L::NQ + NT - 1) / NT;
    float qv0[KQ], qv1[KQ];
    auto load_q = [&](int p) {
        const int pc = clampi(p, 0, mx - 1);
        const int jx = node_of<R>(pc);
#pragma unroll
        for (int k = 0; k < KQ; ++k) {
            const int i = threadIdx.x + k * NT;
            if (i < 3 * L::NQ) {
                const int c = i / L::NQ;
                const int r = i - c * L::NQ;
                const int qz = r % L::NQZ, qy = r / L::NQZ;
                const int gy = min(qly + qy, a.ny - 1), gz = min(qlz + qz, a.nz - 1);
                const uint32_t off = static_cast<uint32_t>(c * nnod + gy * a.nz + gz) * 4u;
                const uint32_t nplane4 = static_cast<uint32_t>(a.ny * a.nz) * 4u;
                qv0[k] = bload(rY, off, static_cast<uint32_t>(jx) * nplane4);
                qv1[k] = bload(rY, off, static_cast<uint32_t>(jx + 1) * nplane4);
            }
        }
    };
    auto store_q = [&](int p) {
        const int pc = clampi(p, 0, mx - 1);
        const double w1 = w1_of<R>(pc), w0 = 1.0 - w1;
#pragma unroll
        for (int k = 0; k < KQ; ++k) {
            const int i = threadIdx.x + k * NT;
            if (i < 3 * L::NQ)
                sQ[i] = w0 * static_cast<double>(qv0[k]) + w1 * static_cast<double>(qv1[k]);
        }
    };
    auto build_q = [&](int p) {
        load_q(p);
        store_q(p);
    };

    // warp at in-plane position (gy, gz) (clamped into the domain) of plane p
    // (clamped), from the x-interpolated node plane
    auto warp_at = [&](int pc, int gy, int gz, float* dT) -> float {
        const int jy = node_of<R>(gy), jz = node_of<R>(gz);
        const double wy1 = w1_of<R>(gy), wz1 = w1_of<R>(gz);
        const double wy0 = 1.0 - wy1, wz0 = 1.0 - wz1;
        const int q = (jy - qly) * L::NQZ + (jz - qlz);
        double yh[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double* Q = sQ + c * L::NQ + q;
            const double c0 = wz0 * Q[0] + wz1 * Q[1];
            const double c1 = wz0 * Q[L::NQZ] + wz1 * Q[L::NQZ + 1];
            yh[c] = wy0 * c0 + wy1 * c1;
        }
        // continuous template index y_hat / h - 1/2; a power-of-two spacing has
        // an exact reciprocal, any other is divided (correctly rounded)
        int i0[3];
        float f[3], s[3];
        const double hh[3] = {a.hx, a.hy, a.hz};
        const double ih[3] = {a.ihx, a.ihy, a.ihz};
        const int mm[3] = {mx, my, mz};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double xi = POW2 ? fma(yh[d], ih[d], -0.5) : yh[d] / hh[d] - 0.5;
            // clamped into [0, m - 1] (a NaN goes to 0); inside the domain iff
            // unchanged.  On [0, m - 1] the floor is the truncation, and the
            // last cell is m - 2 (the fraction reaches 1 at the far end).
            const double xc = fmin(fmax(xi, 0.0), static_cast<double>(mm[d] - 1));
            s[d] = xc == xi ? 1.0f : 0.0f;
            const int i = min(static_cast<int>(xc), mm[d] - 2);
            i0[d] = i;
            f[d] = static_cast<float>(xc - static_cast<double>(i));
        }
        (void)pc;
        const uint32_t tb = static_cast<uint32_t>(i0[0] * sxT + i0[1] * mz + i0[2]) * 4u;
        const uint32_t row4 = static_cast<uint32_t>(mz) * 4u;
        const float2 t00 = bload2(rT, tb, 0u), t01 = bload2(rT, tb, row4);
        const float2 t10 = bload2(rT, tb, plane4), t11 = bload2(rT, tb, plane4 + row4);
        const float v000 = t00.x, v001 = t00.y, v010 = t01.x, v011 = t01.y;
        const float v100 = t10.x, v101 = t10.y, v110 = t11.x, v111 = t11.y;
        const float qx = 1.0f - f[0], qy = 1.0f - f[1], qz = 1.0f - f[2];
        const float c00 = fmaf(f[2], v001, qz * v000), c01 = fmaf(f[2], v011, qz * v010);
        const float c10 = fmaf(f[2], v101, qz * v100), c11 = fmaf(f[2], v111, qz * v110);
        const float c0 = fmaf(f[1], c01, qy * c00), c1 = fmaf(f[1], c11, qy * c10);
        if (GRAD && dT != nullptr) {
            const float d0 = c01 - c00, d1 = c11 - c10;
            const float e00 = v001 - v000, e01 = v011 - v010, e10 = v101 - v100,
                        e11 = v111 - v110;
            dT[0] = (c1 - c0) * (s[0] * a.fihx);
            dT[1] = fmaf(f[0], d1, qx * d0) * (s[1] * a.fihy);
            const float ez0 = fmaf(f[1], e01, qy * e00), ez1 = fmaf(f[1], e11, qy * e10);
            dT[2] = fmaf(f[0], ez1, qx * ez0) * (s[2] * a.fihz);
        }
        return fmaf(f[0], c1, qx * c0);
    };

    // dT of the last three warped planes: dTw is written by W, dT2 (two steps
    // old) is read by E; the registers rotate at the end of every step
    float dTw[L::KP][3], dT1[L::KP][3], dT2[L::KP][3];
    float acc0[L::KO], acc1[L::KO];
#pragma unroll
    for (int o = 0; o < L::KO; ++o) acc0[o] = acc1[o] = 0.0f;
    int jA = jx_first;
    double dsum = 0.0;
    float* part = a.part + static_cast<int64_t>(tile) * 3 * (CX / R + 1) * L::PY * L::PZ;
    const int NPc = (CX / R + 1) * L::PY * L::PZ;

    auto flush = [&](int j, const float* acc) {
        const int lx = j - jx_first;
        if (lx < 0 || lx > CX / R) return;
#pragma unroll
        for (int o = 0; o < L::KO; ++o) {
            const int i = threadIdx.x + o * NT;
            if (i < L::NOUT) {
                const int c = i / (L::PY * L::PZ);
                const int r = i - c * (L::PY * L::PZ);
                part[c * NPc + lx * (L::PY * L::PZ) + r] = acc[o];
            }
        }
    };

    build_q(x0 - 2);
    __syncthreads();

    auto step = [&](const int k) {
        const int S = k % 3;  // LDS slot of the plane warped in this step
        // ---------------- W: warp plane pw, stage R of plane pw - 1 --------
        const int pw = x0 - 2 + k;
        const int pwc = clampi(pw, 0, mx - 1);
        float* Ty = sTy + S * L::NH2;
        const bool wgrad = GRAD && pw >= x0 && pw < xend;
#pragma unroll
        for (int kk = 0; kk < L::KP; ++kk) {
            const int t = threadIdx.x + kk * NT;
            const int ly = t / TZ, lz = t % TZ;
            const int gy = min(y0 + ly, my - 1), gz = min(z0 + lz, mz - 1);
            Ty[(ly + 2) * L::H2Z + (lz + 2)] = warp_at(pwc, gy, gz, wgrad ? dTw[kk] : nullptr);
        }
        for (int s = threadIdx.x; s < L::NRING2; s += NT) {
            int by, bz;
            if (s < 4 * L::H2Z) {
                const int row = s / L::H2Z;
                by = row < 2 ? row : TY + row;
                bz = s - row * L::H2Z;
            } else {
                const int q = s - 4 * L::H2Z;
                const int col = q & 3;
                by = 2 + (q >> 2);
                bz = col < 2 ? col : TZ + col;
            }
            const int gy = clampi(y0 - 2 + by, 0, my - 1), gz = clampi(z0 - 2 + bz, 0, mz - 1);
            Ty[by * L::H2Z + bz] = warp_at(pwc, gy, gz, nullptr);
        }
        const int pv = pw - 1;
        const bool vok = pv >= max(x0 - 1, 0) && pv <= min(x0 + CX, mx - 1);
        // prefetch for the next phases: node values of the next x-interpolated
        // plane, and the x neighbours of R at this thread's V positions
        if (k + 1 < nstep) load_q(pw + 1);
        float rxm[L::KP + 1], rxp[L::KP + 1];
        if (vok) {
            const uint32_t sm = static_cast<uint32_t>(max(pv - 1, 0)) * plane4;
            const uint32_t sp = static_cast<uint32_t>(min(pv + 1, mx - 1)) * plane4;
#pragma unroll
            for (int kk = 0; kk <= L::KP; ++kk) {
                int b1y, b1z;
                if (kk < L::KP) {
                    const int t = threadIdx.x + kk * NT;
                    b1y = t / TZ + 1;
                    b1z = t % TZ + 1;
                } else {
                    ring1_pos(min(static_cast<int>(threadIdx.x), L::NRING1 - 1), b1y, b1z);
                }
                const int cy = clampi(y0 - 1 + b1y, 0, my - 1), cz = clampi(z0 - 1 + b1z, 0, mz - 1);
                const uint32_t off = static_cast<uint32_t>(cy * mz + cz) * 4u;
                rxm[kk] = bload(rR, off, sm);
                rxp[kk] = bload(rR, off, sp);
            }
        }
        if (vok) {
            const uint32_t s0 = static_cast<uint32_t>(pv) * plane4;
            for (int i = threadIdx.x; i < L::NH2; i += NT) {
                const int by = i / L::H2Z, bz = i - by * L::H2Z;
                const int gy = clampi(y0 - 2 + by, 0, my - 1), gz = clampi(z0 - 2 + bz, 0, mz - 1);
                sR[i] = bload(rR, static_cast<uint32_t>(gy * mz + gz) * 4u, s0);
            }
        }
        __syncthreads();

        // ---------------- V: NGF on plane pv ------------------------------
        if (vok) {
            const float* Tm = sTy + ((S + 1) % 3) * L::NH2;  // plane pv - 1 (slot of k - 2)
            const float* T0 = sTy + ((S + 2) % 3) * L::NH2;  // plane pv     (slot of k - 1)
            const float* Tp = Ty;                            // plane pv + 1 (slot of k)
            const bool dtile = pv >= x0 && pv < xend;
            float* Vx = sVx + (pv % 3) * L::NI;
            float* Vy = sVy + (pv & 1) * (L::H1Y * TZ);
            float* Vz = sVz + (pv & 1) * (TY * L::H1Z);
            auto ngf_at = [&](int b1y, int b1z, bool inner, float rm, float rp) {
                const int gy = y0 - 1 + b1y, gz = z0 - 1 + b1z;
                const int cy = clampi(gy, 0, my - 1), cz = clampi(gz, 0, mz - 1);
                const int p = (cy - y0 + 2) * L::H2Z + (cz - z0 + 2);
                const float tau = a.tau, rho = a.rho;
                const float gTx = (Tp[p] - Tm[p]) * a.i2hx;
                const float gTy = (T0[p + L::H2Z] - T0[p - L::H2Z]) * a.i2hy;
                const float gTz = (T0[p + 1] - T0[p - 1]) * a.i2hz;
                const float gRx = (rp - rm) * a.i2hx;
                const float gRy = (sR[p + L::H2Z] - sR[p - L::H2Z]) * a.i2hy;
                const float gRz = (sR[p + 1] - sR[p - 1]) * a.i2hz;
                const float aa = fmaf(gTx, gTx, fmaf(gTy, gTy, fmaf(gTz, gTz, tau * tau)));
                const float bb = fmaf(gRx, gRx, fmaf(gRy, gRy, fmaf(gRz, gRz, rho * rho)));
                const float ab = fmaf(gTx, gRx, fmaf(gTy, gRy, fmaf(gTz, gRz, tau * rho)));
                const float iaa = __builtin_amdgcn_rcpf(aa), ibb = __builtin_amdgcn_rcpf(bb);
                if (inner && dtile && gy < my && gz < mz) {
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
                    if (gy != cy) vy = -vy;  // mirrored ghost of the y adjoint stencil
                    if (gz != cz) vz = -vz;
                    const int hy = (b1y == 0 || b1y == TY + 1), hz = (b1z == 0 || b1z == TZ + 1);
                    if (!hy && !hz) Vx[(b1y - 1) * TZ + (b1z - 1)] = vx;
                    if (!hz) Vy[b1y * TZ + (b1z - 1)] = vy;
                    if (!hy) Vz[(b1y - 1) * L::H1Z + b1z] = vz;
                }
            };
#pragma unroll
            for (int kk = 0; kk < L::KP; ++kk) {
                const int t = threadIdx.x + kk * NT;
                ngf_at(t / TZ + 1, t % TZ + 1, true, rxm[kk], rxp[kk]);
            }
            if (GRAD && threadIdx.x < L::NRING1) {
                int b1y, b1z;
                ring1_pos(threadIdx.x, b1y, b1z);
                ngf_at(b1y, b1z, false, rxm[L::KP], rxp[L::KP]);
            }
        }
        if (!GRAD) {
            __syncthreads();
            if (k + 1 < nstep) store_q(pw + 1);
            __syncthreads();
            return;
        }
        __syncthreads();

        // ---------------- E: adjoint on plane pe --------------------------
        const int pe = pw - 2;
        const bool eok = pe >= x0 && pe < xend;
        if (eok) {
            const float* V0 = sVx + (pe % 3) * L::NI;
            const float* Vm = pe - 1 >= 0 ? sVx + ((pe + 2) % 3) * L::NI : nullptr;
            const float* Vp = pe + 1 <= mx - 1 ? sVx + ((pe + 1) % 3) * L::NI : nullptr;
            const float* Vy = sVy + (pe & 1) * (L::H1Y * TZ);
            const float* Vz = sVz + (pe & 1) * (TY * L::H1Z);
#pragma unroll
            for (int kk = 0; kk < L::KP; ++kk) {
                const int t = threadIdx.x + kk * NT;
                const int ly = t / TZ, lz = t % TZ;
                const float vxm = Vm ? Vm[t] : -V0[t];
                const float vxp = Vp ? Vp[t] : -V0[t];
                const float ex = vxm - vxp;
                const float ey = Vy[ly * TZ + lz] - Vy[(ly + 2) * TZ + lz];
                const float ez = Vz[ly * L::H1Z + lz] - Vz[ly * L::H1Z + lz + 2];
                const bool in = (y0 + ly < my) && (z0 + lz < mz);
                const float e = in ? fmaf(ex, a.i2hx, fmaf(ey, a.i2hy, ez * a.i2hz)) : 0.0f;
                sG[t] = e * dT2[kk][0];  // dT of plane pe, warped two steps ago
                sG[L::NI + t] = e * dT2[kk][1];
                sG[2 * L::NI + t] = e * dT2[kk][2];
            }
        }
        __syncthreads();

        // ---------------- Z: P^T along z ----------------------------------
        // node nz of the tile collects voxels R(nz-1) .. R(nz+1)-1 with the
        // weights (2k+1)/(2R) rising then falling (the two halves of a cell)
        const int jz0 = z0 / R, jy0 = y0 / R;
        if (eok) {
            for (int i = threadIdx.x; i < L::GZ; i += NT) {
                const int nz = i % L::PZ;
                const float* g = sG + (i / L::PZ) * TZ;  // (c, ly) row
                float acc = 0.0f;
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    // voxel R(nz-1)+k: node nz is its upper node (weight w1)
                    const int lz = R * (nz - 1) + k;
                    if (lz >= 0) acc = fmaf((2 * k + 1) * (0.5f / R), g[lz], acc);
                    // voxel R nz + k: node nz is its lower node (weight w0)
                    const int lz2 = R * nz + k;
                    if (lz2 < TZ) acc = fmaf(1.0f - (2 * k + 1) * (0.5f / R), g[lz2], acc);
                }
                sGz[i] = acc;
            }
        }
        __syncthreads();

        // ---------------- Y: P^T along y, then x into the accumulators -----
        if (eok) {
            const int jx = node_of<R>(pe);
            const float wx1 = w1_of<R>(pe), wx0 = 1.0f - wx1;
            if (jx > jA) {  // node plane jA has all its image planes: write it
                flush(jA, acc0);
#pragma unroll
                for (int o = 0; o < L::KO; ++o) {
                    acc0[o] = acc1[o];
                    acc1[o] = 0.0f;
                }
                jA += 1;
            }
#pragma unroll
            for (int o = 0; o < L::KO; ++o) {
                const int i = threadIdx.x + o * NT;
                if (i < L::NOUT) {
                    const int nz = i % L::PZ;
                    const int ny = (i / L::PZ) % L::PY;
                    const int c = i / (L::PZ * L::PY);
                    const float* gz = sGz + c * TY * L::PZ + nz;
                    float v = 0.0f;
#pragma unroll
                    for (int k = 0; k < R; ++k) {
                        const int ly = R * (ny - 1) + k;
                        if (ly >= 0) v = fmaf((2 * k + 1) * (0.5f / R), gz[ly * L::PZ], v);
                        const int ly2 = R * ny + k;
                        if (ly2 < TY) v = fmaf(1.0f - (2 * k + 1) * (0.5f / R), gz[ly2 * L::PZ], v);
                    }
                    acc0[o] = fmaf(wx0, v, acc0[o]);
                    acc1[o] = fmaf(wx1, v, acc1[o]);
                }
            }
        }
        if (k + 1 < nstep) store_q(pw + 1);  // sG is no longer read: Q may overwrite it
#pragma unroll
        for (int kk = 0; kk < L::KP; ++kk)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                dT2[kk][c] = dT1[kk][c];
                dT1[kk][c] = dTw[kk][c];
            }
        __syncthreads();
    };

    for (int k = 0; k < nstep; ++k) step(k);
    if (GRAD) {
        flush(jA, acc0);
        flush(jA + 1, acc1);
    }
    const double dt = [&] {
        double v = wave_sum(dsum);
        const int w = threadIdx.x >> 6;
        __syncthreads();
        if ((threadIdx.x & 63) == 0) red[w] = v;
        __syncthreads();
        if constexpr (NT == 256)
            return (red[0] + red[1]) + (red[2] + red[3]);
        else
            return ((red[0] + red[1]) + (red[2] + red[3])) +
                   ((red[4] + red[5]) + (red[6] + red[7]));
    }();
    if (threadIdx.x == 0) a.dpart[tile] = dt;
}

// The 16 x 32 tile needs 36 KiB of LDS, so up to four workgroups fit a CU;
// its registers are held to four waves per SIMD (128 VGPRs, no spills).  The
// 32 x 32 tile (512 threads, 68 KiB) fits two workgroups, also four waves
// per SIMD.  The 16 x 64 tile is limited to two workgroups per CU by LDS.
template <int TY, int TZ, int R, bool GRAD, bool POW2>
__global__ __launch_bounds__((march_threads<TY, TZ>()), TZ == 32 ? 4 : 2) void k_image_march(
    ImagePassArgs a, int CX) {
    if (a.gate && *a.gate == kOpNone) return;
    march_body<TY, TZ, R, GRAD, POW2>(a, CX, blockIdx.x);
}

// each pair's chunk length is its own (a.cx).  The pair and block indices
// are uniform over the workgroup: taken as such, the pair's arguments load
// into scalar registers and the kernel needs no more vector registers than
// the single-pair one (no spills).
template <int TY, int TZ, int R, bool POW2>
__global__ __launch_bounds__((march_threads<TY, TZ>()), TZ == 32 ? 4 : 2) void k_image_march_batch(
    const ImagePassArgs* args, const BlockRef* blk) {
    const BlockRef e = blk[blockIdx.x];
    const int pair = __builtin_amdgcn_readfirstlane(e.pair);
    if (pair < 0) return;
    const ImagePassArgs a = args[pair];
    if (a.gate && *a.gate == kOpNone) return;
    march_body<TY, TZ, R, true, POW2>(a, __builtin_amdgcn_readfirstlane(a.cx),
                                      __builtin_amdgcn_readfirstlane(e.block));
}

template <int TY, int TZ, int R>
void launch_march_batch_t(const ImagePassArgs* args, const BlockRef* blk, int nblk, bool pow2,
                          hipStream_t s) {
    using L = March<TY, TZ, R>;
    const size_t lds = sizeof(float) * L::LDS_FLOATS;
    if (pow2)
        hipLaunchKernelGGL((k_image_march_batch<TY, TZ, R, true>), dim3(nblk), dim3(L::NT),
                           lds, s, args, blk);
    else
        hipLaunchKernelGGL((k_image_march_batch<TY, TZ, R, false>), dim3(nblk), dim3(L::NT),
                           lds, s, args, blk);
}

template <int TY, int TZ, int R>
void launch_march_t(const ImagePassArgs& a, int cx, hipStream_t s) {
    using L = March<TY, TZ, R>;
    const int blocks = a.ntx * a.nty * a.ntz;
    const size_t lds = sizeof(float) * L::LDS_FLOATS;
    // the spacing decides at compile time how the warp index is formed
    if (a.want_grad) {
        if (a.pow2h)
            hipLaunchKernelGGL((k_image_march<TY, TZ, R, true, true>), dim3(blocks),
                               dim3(L::NT), lds, s, a, cx);
        else
            hipLaunchKernelGGL((k_image_march<TY, TZ, R, true, false>), dim3(blocks),
                               dim3(L::NT), lds, s, a, cx);
    } else {
        if (a.pow2h)
            hipLaunchKernelGGL((k_image_march<TY, TZ, R, false, true>), dim3(blocks),
                               dim3(L::NT), lds, s, a, cx);
        else
            hipLaunchKernelGGL((k_image_march<TY, TZ, R, false, false>), dim3(blocks),
                               dim3(L::NT), lds, s, a, cx);
    }
}

}  // namespace

// gradient form only (the batched rounds always want the gradient)
void launch_image_march_batch(const ImagePassArgs* args, const BlockRef* blk, int nblk,
                              int ratio, int variant, bool pow2, hipStream_t s) {
    if (nblk <= 0) return;
    const int ty = march_ty(variant), tz = march_tz(variant);
    if (ty == 32) {
        if (ratio == 2)
            launch_march_batch_t<32, 32, 2>(args, blk, nblk, pow2, s);
        else if (ratio == 4)
            launch_march_batch_t<32, 32, 4>(args, blk, nblk, pow2, s);
    } else if (tz == 64) {
        if (ratio == 2)
            launch_march_batch_t<kMY, 64, 2>(args, blk, nblk, pow2, s);
        else if (ratio == 4)
            launch_march_batch_t<kMY, 64, 4>(args, blk, nblk, pow2, s);
    } else {
        if (ratio == 2)
            launch_march_batch_t<kMY, 32, 2>(args, blk, nblk, pow2, s);
        else if (ratio == 4)
            launch_march_batch_t<kMY, 32, 4>(args, blk, nblk, pow2, s);
    }
}

namespace {
template <int TY, int TZ>
int march_per_cu() {
    using L = March<TY, TZ, 2>;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_image_march<TY, TZ, 2, true, true>,
                                                     L::NT, sizeof(float) * L::LDS_FLOATS) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return per_cu;
}
}  // namespace

int image_march_slots(int ty, int tz) {
    // occupancy per CU, queried once per device and tile (the ratio-2
    // instance stands for both ratios: same launch bounds, same LDS)
    static std::atomic<int> cache[16][3];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) dev = 0;
    const int form = ty == 32 ? 2 : (tz == 64 ? 1 : 0);
    std::atomic<int>& slot = cache[dev & 15][form];
    int v = slot.load();
    if (v > 0) return v;
    const int per_cu = form == 2 ? march_per_cu<32, 32>()
                                 : (form == 1 ? march_per_cu<kMY, 64>() : march_per_cu<kMY, 32>());
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        cus = 256;
    (void)hipGetLastError();
    v = per_cu * cus;
    slot.store(v);
    return v;
}

void launch_image_march(const ImagePassArgs& a, int ratio, int ty, int tz, int cx,
                        hipStream_t s) {
    if (ty == 32) {
        if (ratio == 2)
            launch_march_t<32, 32, 2>(a, cx, s);
        else if (ratio == 4)
            launch_march_t<32, 32, 4>(a, cx, s);
    } else if (tz == 64) {
        if (ratio == 2)
            launch_march_t<kMY, 64, 2>(a, cx, s);
        else if (ratio == 4)
            launch_march_t<kMY, 64, 4>(a, cx, s);
    } else {
        if (ratio == 2)
            launch_march_t<kMY, 32, 2>(a, cx, s);
        else if (ratio == 4)
            launch_march_t<kMY, 32, 4>(a, cx, s);
    }
}

}  // namespace ngf
