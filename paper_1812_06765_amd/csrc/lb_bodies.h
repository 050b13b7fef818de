// Device bodies of the L-BFGS kernels (Sec. 2.1: L-BFGS after Nocedal,
// 1980), shared by the single-pair kernels and their batched forms.
// See k_lbfgs.hip for the method.
#pragma once

#include <math.h>

#include "../../include/ngfreg.h"
#include "ngf_internal.h"

namespace ngf {

namespace {

constexpr int kDots = 6 * kSlots + 6;

// inner products formed per update
static_assert(kDots <= 64, "one lane per inner product in the Gram update");

constexpr int kLbBlocks = 768;

// Whether the L-BFGS vector passes of a level with n unknowns stream the
// stored pairs and the direction past the last-level cache: from 4 Mi
// unknowns on, the pairs alone fill a large part of it and would push out
// the level's images, which every image pass reads again.
__device__ inline bool lb_streams(int64_t n) { return n >= (int64_t{1} << 22); }

// 16-byte loads and stores of the vector passes.  With NT the streams that
// nothing reads again soon (the stored pairs, the direction, and in the
// history update the last reads of y, g and their trial values) bypass the
// last-level cache, which then keeps the level's images for the image pass.
typedef float lb_f4 __attribute__((ext_vector_type(4)));
template <bool NT>
__device__ inline float4 lb_ld4(const float* p, int64_t q) {
    if constexpr (NT) {
        const lb_f4 v = __builtin_nontemporal_load(reinterpret_cast<const lb_f4*>(p) + q);
        return make_float4(v.x, v.y, v.z, v.w);
    } else {
        return reinterpret_cast<const float4*>(p)[q];
    }
}
template <bool NT>
__device__ inline void lb_st4(float* p, int64_t q, float4 v) {
    if constexpr (NT) {
        lb_f4 w;
        w.x = v.x;
        w.y = v.y;
        w.z = v.z;
        w.w = v.w;
        __builtin_nontemporal_store(w, reinterpret_cast<lb_f4*>(p) + q);
    } else {
        reinterpret_cast<float4*>(p)[q] = v;
    }
}

__device__ inline double lb_wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

__device__ inline void lb_init_one(LbState* st, int mem, double hmin, const double* jds,
                                   int max_iter, int early_stop, double tol) {
    LbCtl& c = st->ctl;
    c.op = kOpNone;
    c.phase = kPhNeedDir;
    c.halvings = 0;
    c.iters = 0;
    c.evals = 1;
    c.info = NGF_INFO_MAX_ITER;
    c.max_iter = max_iter;
    c.early_stop = early_stop;
    c.t = 1.0;
    c.tol = tol;
    c.J = jds[0];
    c.gmax = jds[3];
    st->count = 0;
    st->free_slot = 0;
    st->mem = mem;
    st->hmin = hmin;
    for (int i = 0; i < kSlots; ++i) st->order[i] = -1;
    st->J = jds[0];
    st->D = jds[1];
    st->S = jds[2];
    st->gmax = jds[3];
    st->gnorm2 = jds[4];
    st->gtd = 0.0;
    st->flags = 0.0;
    st->count_d = 0.0;
    for (int i = 0; i < kBasis * kBasis; ++i) st->G[i] = 0.0;
    for (int i = 0; i < kBasis; ++i) st->coef[i] = 0.0;
    st->G[kBasisG * kBasis + kBasisG] = jds[4];
    st->reject_all = 0;  // failure injection: set by the host after this kernel
}

// Direction coefficients by the two-loop recursion over the Gram matrix.
// Falls back to the scaled steepest-descent step (and drops the memory) when
// there is no pair or the recursion does not give a descent direction.
// The current point's J, max |g| and |g|^2 are taken from the state, where
// k_lb_init and k_lb_gram_update put them.  g^T d also goes to jds[5], which
// the next evaluation's reduction leaves alone (it writes jds[0..4]).
// Working set of the recursion, staged in LDS by the calling kernel: the
// recursion is a chain of dependent reads and small-array updates, far
// cheaper from LDS than from L2 or from scratch memory.
struct SolveLds {
    double G[kBasis * kBasis];
    double q[kBasis];
    double al[kSlots];
    int order[kSlots];
};

__device__ inline void lb_stage(const LbState* st, SolveLds& w) {
    for (int i = threadIdx.x; i < kBasis * kBasis; i += blockDim.x) w.G[i] = st->G[i];
    for (int i = threadIdx.x; i < kSlots; i += blockDim.x) w.order[i] = st->order[i];
    __syncthreads();
}

// Sum over the 64 lanes of a wave by a butterfly: every lane ends with the
// same value (each step adds a + b and b + a, which round alike).
__device__ inline double lb_wave_allsum(double v) {
    for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// The recursion on one wave: lane l < kBasis holds the coefficient q_l of
// basis vector l, each inner product q^T G e_i is a wave sum, and the scalars
// of the recursion (every lane computes them alike) stay in registers; lane k
// keeps alpha_k for the second loop.  The g^T g entry of G refers to the
// current gradient: it is read as such here and set in the state.  Called by
// every lane of the block's first wave.
__device__ inline void lb_solve_wave(LbState* st, double* jds, SolveLds& w) {
    const int l = threadIdx.x & 63;
    const double* G = w.G;
    const double gn2 = st->gnorm2;
    auto Gat = [&](int i, int j) {
        return (i == kBasisG && j == kBasisG) ? gn2 : G[i * kBasis + j];
    };
    auto row_dot = [&](double q, int i) {  // sum_l q_l G(i, l)
        return lb_wave_allsum(l < kBasis ? q * Gat(i, l) : 0.0);
    };
    const double gmax = st->gmax, hmin = st->hmin;
    int count = st->count;
    if (l == 0) st->G[kBasisG * kBasis + kBasisG] = gn2;
    if (!(gmax > 0.0)) {
        if (l == 0) {
            st->flags = 2.0;
            st->gtd = 0.0;
            jds[5] = 0.0;
        }
        if (l < kBasis) st->coef[l] = 0.0;
        return;
    }
    double flags = 0.0, gtd = 0.0, q = 0.0;
    if (count > 0) {
        q = l == kBasisG ? 1.0 : 0.0;
        double al = 0.0;
        for (int k = count - 1; k >= 0; --k) {
            const int si = w.order[k], ti = kSlots + si;
            const double a = row_dot(q, si) / Gat(si, ti);
            if (l == k) al = a;
            if (l == ti) q -= a;
        }
        const int sn = w.order[count - 1], tn = kSlots + sn;
        q *= Gat(sn, tn) / Gat(tn, tn);
        for (int k = 0; k < count; ++k) {
            const int si = w.order[k], ti = kSlots + si;
            const double b = row_dot(q, ti) / Gat(si, ti);
            const double a = __shfl(al, k, 64);
            if (l == si) q += a - b;
        }
        q = -q;  // the coefficients of d
        gtd = row_dot(q, kBasisG);
        if (!(gtd < 0.0)) {
            count = 0;
            flags = 1.0;
        }
    }
    if (count == 0) {
        if (l == 0) {
            st->count = 0;
            st->free_slot = 0;
        }
        if (l < kSlots) st->order[l] = -1;
        const double scale = hmin / gmax;
        q = l == kBasisG ? -scale : 0.0;
        gtd = -scale * gn2;
    }
    if (l < kBasis) st->coef[l] = q;
    if (l == 0) {
        st->gtd = gtd;
        st->flags = flags;
        st->count_d = static_cast<double>(count);
        jds[5] = gtd;  // read by the host with the trial's J in one copy
    }
}

// d = sum_l coef_l b_l over the active basis; yt = y + d.  Four elements per
// thread and iteration (16-byte loads), then a scalar tail.  The pairs are
// visited in a loop (two history streams at a time): unrolling it over all
// pairs measured slower.
template <bool NT>
__device__ __forceinline__ void lb_combine_body(const LbState* st,
                                                const float* __restrict__ hist, int64_t ld,
                                                int64_t n, const float* __restrict__ y,
                                                const float* __restrict__ g,
                                                float* __restrict__ d, float* __restrict__ yt,
                                                int block, int nblocks) {
    __shared__ double cs[kSlots], ct[kSlots];
    __shared__ int sl[kSlots];
    __shared__ double cg;
    __shared__ int cnt;
    if (threadIdx.x == 0) {
        cnt = st->count;
        cg = st->coef[kBasisG];
        for (int k = 0; k < kSlots; ++k) {
            const int s = k < st->count ? st->order[k] : 0;
            sl[k] = s;
            cs[k] = k < st->count ? st->coef[s] : 0.0;
            ct[k] = k < st->count ? st->coef[kSlots + s] : 0.0;
        }
    }
    __syncthreads();
    const int count = cnt;
    const int64_t n4 = n >> 2;
    const int64_t stride = static_cast<int64_t>(nblocks) * kThreads;
    for (int64_t q = block * static_cast<int64_t>(kThreads) + threadIdx.x; q < n4;
         q += stride) {
        const float4 gv = reinterpret_cast<const float4*>(g)[q];
        double v0 = cg * gv.x, v1 = cg * gv.y, v2 = cg * gv.z, v3 = cg * gv.w;
        for (int k = 0; k < count; ++k) {
            const float* sk = hist + (2 * static_cast<int64_t>(sl[k])) * ld;
            const float4 a = lb_ld4<NT>(sk, q);
            const float4 b = lb_ld4<NT>(sk + ld, q);
            v0 += cs[k] * a.x + ct[k] * b.x;
            v1 += cs[k] * a.y + ct[k] * b.y;
            v2 += cs[k] * a.z + ct[k] * b.z;
            v3 += cs[k] * a.w + ct[k] * b.w;
        }
        const float4 yv = reinterpret_cast<const float4*>(y)[q];
        const float4 dv = make_float4(static_cast<float>(v0), static_cast<float>(v1),
                                      static_cast<float>(v2), static_cast<float>(v3));
        lb_st4<NT>(d, q, dv);
        reinterpret_cast<float4*>(yt)[q] =
            make_float4(yv.x + dv.x, yv.y + dv.y, yv.z + dv.z, yv.w + dv.w);
    }
    for (int64_t i = 4 * n4 + block * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
         i += stride) {
        double v = cg * static_cast<double>(g[i]);
        for (int k = 0; k < count; ++k) {
            const float* sk = hist + (2 * static_cast<int64_t>(sl[k])) * ld;
            v += cs[k] * static_cast<double>(sk[i]) + ct[k] * static_cast<double>(sk[ld + i]);
        }
        const float df = static_cast<float>(v);
        d[i] = df;
        yt[i] = y[i] + df;
    }
}

__device__ __forceinline__ void lb_axpy_body(const float* __restrict__ y,
                                                      const float* __restrict__ d, float t,
                                                      float* __restrict__ yt, int64_t n, int block, int nblocks) {
    const int64_t n4 = n >> 2;
    const int64_t stride = static_cast<int64_t>(nblocks) * kThreads;
    for (int64_t q = block * static_cast<int64_t>(kThreads) + threadIdx.x; q < n4;
         q += stride) {
        const float4 a = reinterpret_cast<const float4*>(y)[q];
        const float4 b = reinterpret_cast<const float4*>(d)[q];
        reinterpret_cast<float4*>(yt)[q] =
            make_float4(fmaf(t, b.x, a.x), fmaf(t, b.y, a.y), fmaf(t, b.z, a.z),
                        fmaf(t, b.w, a.w));
    }
    for (int64_t i = 4 * n4 + block * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
         i += stride)
        yt[i] = fmaf(t, d[i], y[i]);
}

// Pass over the elements for C stored pairs (a compile-time count, so that
// only 6 C + 6 float64 accumulators are live).  With ACCEPT, the accepted
// trial point also replaces the current one (y = yt, g = gt), each element
// by the thread that has just read it.
template <bool ACCEPT, int C, bool NT>
__device__ __forceinline__ void lb_dots_pass(const int* sl, int fs, float* __restrict__ hist,
                                             int64_t ld, int64_t n, float* y,
                                             const float* __restrict__ yt, float* g,
                                             const float* __restrict__ gt,
                                             double* __restrict__ dotpart, int block,
                                             int nblocks, double (*sh)[kDots]) {
    constexpr int kA = 6 * C + 6;  // live accumulators; self products last
    double acc[kA];
#pragma unroll
    for (int j = 0; j < kA; ++j) acc[j] = 0.0;
    float* sn = hist + (2 * static_cast<int64_t>(fs)) * ld;
    float* tn = sn + ld;
    auto add = [&](float s, float t, float gn, const float* a, const float* b) {
        const double sd = s, td = t, gd = gn;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const double av = a[k], bv = b[k];
            acc[6 * k + 0] += sd * av;
            acc[6 * k + 1] += sd * bv;
            acc[6 * k + 2] += td * av;
            acc[6 * k + 3] += td * bv;
            acc[6 * k + 4] += gd * av;
            acc[6 * k + 5] += gd * bv;
        }
        acc[6 * C + 0] += sd * sd;
        acc[6 * C + 1] += sd * td;
        acc[6 * C + 2] += sd * gd;
        acc[6 * C + 3] += td * td;
        acc[6 * C + 4] += td * gd;
        acc[6 * C + 5] += gd * gd;
    };
    const int64_t n4 = n >> 2;
    const int64_t stride = static_cast<int64_t>(nblocks) * kThreads;
    const float* hk[C > 0 ? C : 1];
#pragma unroll
    for (int k = 0; k < C; ++k) hk[k] = hist + (2 * static_cast<int64_t>(sl[k])) * ld;
    for (int64_t q = block * static_cast<int64_t>(kThreads) + threadIdx.x; q < n4;
         q += stride) {
        const float4 yv = lb_ld4<NT>(y, q);
        const float4 ytv = lb_ld4<NT>(yt, q);
        const float4 gv = lb_ld4<NT>(g, q);
        const float4 gtv = lb_ld4<NT>(gt, q);
        float4 av[C > 0 ? C : 1], bv[C > 0 ? C : 1];
#pragma unroll
        for (int k = 0; k < C; ++k) {
            av[k] = lb_ld4<NT>(hk[k], q);
            bv[k] = lb_ld4<NT>(hk[k] + ld, q);
        }
        const float4 s = make_float4(ytv.x - yv.x, ytv.y - yv.y, ytv.z - yv.z, ytv.w - yv.w);
        const float4 t = make_float4(gtv.x - gv.x, gtv.y - gv.y, gtv.z - gv.z, gtv.w - gv.w);
        lb_st4<NT>(sn, q, s);
        lb_st4<NT>(tn, q, t);
        if (ACCEPT) {
            reinterpret_cast<float4*>(y)[q] = ytv;
            reinterpret_cast<float4*>(g)[q] = gtv;
        }
        float a0[C > 0 ? C : 1], b0[C > 0 ? C : 1], a1[C > 0 ? C : 1], b1[C > 0 ? C : 1];
        float a2[C > 0 ? C : 1], b2[C > 0 ? C : 1], a3[C > 0 ? C : 1], b3[C > 0 ? C : 1];
#pragma unroll
        for (int k = 0; k < C; ++k) {
            a0[k] = av[k].x;
            a1[k] = av[k].y;
            a2[k] = av[k].z;
            a3[k] = av[k].w;
            b0[k] = bv[k].x;
            b1[k] = bv[k].y;
            b2[k] = bv[k].z;
            b3[k] = bv[k].w;
        }
        add(s.x, t.x, gtv.x, a0, b0);
        add(s.y, t.y, gtv.y, a1, b1);
        add(s.z, t.z, gtv.z, a2, b2);
        add(s.w, t.w, gtv.w, a3, b3);
    }
    for (int64_t i = 4 * n4 + block * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
         i += stride) {
        const float yti = yt[i], gti = gt[i];
        const float s = yti - y[i];
        const float t = gti - g[i];
        sn[i] = s;
        tn[i] = t;
        if (ACCEPT) {
            y[i] = yti;
            g[i] = gti;
        }
        float a[C > 0 ? C : 1], b[C > 0 ? C : 1];
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const float* sk = hist + (2 * static_cast<int64_t>(sl[k])) * ld;
            a[k] = sk[i];
            b[k] = sk[ld + i];
        }
        add(s, t, gti, a, b);
    }
    // wave sums, then the four waves in a fixed order; dots of unused slots are 0
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < kA; ++j) {
        const double v = lb_wave_sum(acc[j]);
        const int o = j < 6 * C ? j : 6 * kSlots + (j - 6 * C);
        if ((threadIdx.x & 63) == 0) sh[w][o] = v;
    }
    for (int o = 6 * C + threadIdx.x; o < 6 * kSlots; o += kThreads)
        sh[0][o] = sh[1][o] = sh[2][o] = sh[3][o] = 0.0;
    __syncthreads();
    for (int j = threadIdx.x; j < kDots; j += kThreads)
        dotpart[static_cast<int64_t>(block) * kDots + j] =
            (sh[0][j] + sh[1][j]) + (sh[2][j] + sh[3][j]);
}

// Forms the new pair s = yt - y, t = gt - g in the free slot and all inner
// products of {s, t, gt} with the stored pairs and with each other.
// Per-block float64 partials: dotpart[block][kDots].  Four elements per
// thread and iteration (16-byte loads), then a scalar tail.
// CMAX: the largest pair count the kernel is built for (the L-BFGS memory
// rounded up to 5 or 8); registers are allocated for the largest case.
template <bool ACCEPT, int CMAX, bool NT>
__device__ __forceinline__ void lb_update_dots_body(const LbState* st,
                                                    float* __restrict__ hist, int64_t ld,
                                                    int64_t n, float* y,
                                                    const float* __restrict__ yt, float* g,
                                                    const float* __restrict__ gt,
                                                    double* __restrict__ dotpart, int block,
                                                    int nblocks) {
    __shared__ int sl[kSlots];
    __shared__ int cnt, fs;
    __shared__ double sh[4][kDots];
    if (threadIdx.x == 0) {
        cnt = st->count;
        fs = st->free_slot;
        for (int k = 0; k < kSlots; ++k) sl[k] = k < st->count ? st->order[k] : 0;
    }
    __syncthreads();
    switch (cnt) {
#define NGF_DOTS_CASE(C)                                                                \
    case C:                                                                             \
        lb_dots_pass<ACCEPT, (C <= CMAX ? C : CMAX), NT>(sl, fs, hist, ld, n, y, yt, g,   \
                                                         gt, dotpart, block, nblocks, sh);  \
        break;
        NGF_DOTS_CASE(0)
        NGF_DOTS_CASE(1)
        NGF_DOTS_CASE(2)
        NGF_DOTS_CASE(3)
        NGF_DOTS_CASE(4)
        NGF_DOTS_CASE(5)
        NGF_DOTS_CASE(6)
        NGF_DOTS_CASE(7)
        NGF_DOTS_CASE(8)
#undef NGF_DOTS_CASE
        default:
            break;
    }
}

// Fixed-order sum of the per-block dot partials, curvature test of the new
// pair, ring update and Gram-matrix update.  The partials are summed by 1024
// threads: thread t adds dot (t mod 64) over the blocks b = t/64, t/64 + 16,
// ..., and the 16 phase sums of each dot are then added in phase order.
constexpr int kGramThreads = 1024;

constexpr int kGramPhases = kGramThreads / 64;

__device__ __forceinline__ void lb_gram_one(LbState* st, const double* dots, const double* jds);

__device__ __forceinline__ void lb_gram_body(LbState* st,
                                                                 const double* dotpart,
                                                                 int nblocks,
                                                                 const double* jds) {
    __shared__ double ph[kGramPhases][64];
    __shared__ double dots[kDots];
    // phase p sums blocks p, p + 16, ...; with fewer than 1024 threads a
    // thread takes several phases (the same sums)
    for (int p = threadIdx.x >> 6; p < kGramPhases; p += blockDim.x >> 6) {
        const int j = threadIdx.x & 63;
        double s = 0.0;
        if (j < kDots) {
            // all loads of a phase in flight at once (768 blocks: 48 each);
            // the additions keep the block order
#pragma unroll 48
            for (int b = p; b < nblocks; b += kGramPhases)
                s += dotpart[static_cast<int64_t>(b) * kDots + j];
        }
        ph[p][j] = s;
    }
    __syncthreads();
    if (threadIdx.x < kDots) {
        double s = 0.0;
        for (int p = 0; p < kGramPhases; ++p) s += ph[p][threadIdx.x];
        dots[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) lb_gram_one(st, dots, jds);
}

// The Gram update itself (one lane): curvature test of the new pair, ring
// update, new entries of G.
__device__ __forceinline__ void lb_gram_one(LbState* st, const double* dots, const double* jds) {
    double* G = st->G;
    const int count = st->count;
    const int fs = st->free_slot;
    const double ss = dots[6 * kSlots + 0], sz = dots[6 * kSlots + 1],
                 sg = dots[6 * kSlots + 2], zz = dots[6 * kSlots + 3],
                 zg = dots[6 * kSlots + 4], gg = dots[6 * kSlots + 5];
    const bool accept = sz > 1e-10 * sqrt(ss) * sqrt(zz);
    auto setg = [&](int i, int j, double v) {
        G[i * kBasis + j] = v;
        G[j * kBasis + i] = v;
    };
    // the gradient row refers to the new gradient from now on
    for (int k = 0; k < count; ++k) {
        const int s = st->order[k];
        setg(kBasisG, s, dots[6 * k + 4]);
        setg(kBasisG, kSlots + s, dots[6 * k + 5]);
    }
    setg(kBasisG, kBasisG, gg);
    if (accept) {
        const int S = fs, T = kSlots + fs;
        for (int k = 0; k < count; ++k) {
            const int s = st->order[k];
            setg(S, s, dots[6 * k + 0]);
            setg(S, kSlots + s, dots[6 * k + 1]);
            setg(T, s, dots[6 * k + 2]);
            setg(T, kSlots + s, dots[6 * k + 3]);
        }
        setg(S, S, ss);
        setg(S, T, sz);
        setg(T, T, zz);
        setg(kBasisG, S, sg);
        setg(kBasisG, T, zg);
        int c = count;
        if (c == st->mem) {  // drop the oldest pair
            for (int k = 1; k < c; ++k) st->order[k - 1] = st->order[k];
            c -= 1;
        }
        st->order[c] = fs;
        st->count = c + 1;
        // next free slot: the lowest slot not in use
        for (int s = 0; s < kSlots; ++s) {
            bool used = false;
            for (int k = 0; k < st->count; ++k) used |= (st->order[k] == s);
            if (!used) {
                st->free_slot = s;
                break;
            }
        }
    }
    st->count_d = static_cast<double>(st->count);
    st->J = jds[0];
    st->D = jds[1];
    st->S = jds[2];
    st->gmax = jds[3];
    st->gnorm2 = jds[4];
}

// ---------------------------------------------------------------------------
// One round of the device-driven level.  Every kernel reads the control block
// first and does nothing when its part of the round does not apply, so a
// round enqueued after the level has ended is a no-op.
// ---------------------------------------------------------------------------


// Start of a round: a new direction (two-loop recursion) after an accepted
// step, or the next halving of the step after a rejected trial.  The tests
// before a new direction are those of one L-BFGS iteration: iteration
// budget, non-finite gradient, zero gradient.
__device__ __forceinline__ void lb_plan_body(LbState* st, double* jds) {
    __shared__ SolveLds w;
    lb_stage(st, w);
    if (threadIdx.x >= 64) return;  // the first wave decides; lane 0 writes
    LbCtl& c = st->ctl;
    const bool lead = threadIdx.x == 0;
    const int phase = c.phase;
    if (phase == kPhDone) {
        if (lead) c.op = kOpNone;
    } else if (phase == kPhNeedDir) {
        const int iters = c.iters, max_iter = c.max_iter;
        const double gmax = c.gmax;
        if (iters >= max_iter) {
            if (lead) lb_finish(c, NGF_INFO_MAX_ITER);
        } else if (!isfinite(gmax)) {
            if (lead) lb_finish(c, NGF_INFO_NONFINITE);
        } else if (gmax == 0.0) {
            if (lead) lb_finish(c, NGF_INFO_CONVERGED);
        } else {
            lb_solve_wave(st, jds, w);
            if (lead) {
                c.t = 1.0;
                c.halvings = 0;
                c.phase = kPhTrial;
                c.op = kOpCombine;
            }
        }
    } else if (lead) {
        c.op = kOpAxpy;  // kPhTrial after a rejection: same d, halved t
    }
}

__device__ __forceinline__ void lb_vec_body(const LbState* st, const float* __restrict__ hist,
                                            int64_t ld, int64_t n, const float* __restrict__ y,
                                            const float* __restrict__ g,
                                            float* __restrict__ d, float* __restrict__ yt,
                                            int block, int nblocks, bool nt) {
    const int op = st->ctl.op;
    if (op == kOpCombine) {
        if (nt)
            lb_combine_body<true>(st, hist, ld, n, y, g, d, yt, block, nblocks);
        else
            lb_combine_body<false>(st, hist, ld, n, y, g, d, yt, block, nblocks);
    } else if (op == kOpAxpy) {
        lb_axpy_body(y, d, static_cast<float>(st->ctl.t), yt, n, block, nblocks);
    }
}

// Gram update for the accepted step, then the stopping tests of the level:
// relative decrease (early stop) and the iteration budget.
__device__ __forceinline__ void lb_accept_gram_body(LbState* st, const double* dotpart,
                                                    int nblocks, const double* jds) {
#pragma clang fp contract(off)
    lb_gram_body(st, dotpart, nblocks, jds);
    if (threadIdx.x == 0) {
        LbCtl& c = st->ctl;
        const double J_old = c.J, J_new = jds[0];
        c.J = J_new;
        c.gmax = jds[3];
        c.iters += 1;
        c.op = kOpNone;
        if (c.early_stop && (J_old - J_new) <= c.tol * (1.0 + fabs(J_old)))
            lb_finish(c, NGF_INFO_CONVERGED);
        else if (c.iters >= c.max_iter)
            lb_finish(c, NGF_INFO_MAX_ITER);
        else
            c.phase = kPhNeedDir;
    }
}

// End of a round and start of the next in one launch: the Gram update and
// stopping tests after an accepted step, then the plan of the next round
// (new direction or next halving).  The same steps, in the same order, as
// the accept and plan kernels launched one after the other; the block's
// barrier makes lane 0's writes to the state visible to the staging of G.
// The state is staged in LDS for the single-lane parts (many dependent
// reads and writes of small fields) and written back once.
__device__ __forceinline__ void lb_gram_plan_body(LbState* st, const double* dotpart,
                                                  int nblocks, double* jds) {
    static_assert(sizeof(LbState) % 8 == 0, "state copied in 8-byte words");
    constexpr int kWords = sizeof(LbState) / 8;
    __shared__ LbState ls;
    {
        const uint64_t* src = reinterpret_cast<const uint64_t*>(st);
        uint64_t* dst = reinterpret_cast<uint64_t*>(&ls);
        for (int i = threadIdx.x; i < kWords; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    if (ls.ctl.phase == kPhAccepted) lb_accept_gram_body(&ls, dotpart, nblocks, jds);
    __syncthreads();
    lb_plan_body(&ls, jds);
    __syncthreads();
    {
        const uint64_t* src = reinterpret_cast<const uint64_t*>(&ls);
        uint64_t* dst = reinterpret_cast<uint64_t*>(st);
        for (int i = threadIdx.x; i < kWords; i += blockDim.x) dst[i] = src[i];
    }
}

}  // namespace

}  // namespace ngf
