// Device body of the final reduction of an evaluation (J = D + alpha S of
// Eq. 1 from the block partials, max |grad J| and |grad J|^2), shared by the
// single-pair kernel and its batched form.
#pragma once

#include "ngf_internal.h"

namespace ngf {

namespace {

// Fixed-order reduction of the per-block partials: thread t combines entries
// t, t + 256, ... in order, each wave folds its 64 lanes by a fixed
// shuffle tree, and thread 0 combines the four wave results in order.
__device__ inline double rd_wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ inline double rd_wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    return v;
}

__device__ __forceinline__ void reduce_body(const ReduceArgs& a) {
    static_assert(kThreads == 256, "four waves");
    __shared__ double sh[4][4];
    double d = 0.0, s = 0.0, m = 0.0, q = 0.0;
#pragma unroll 4
    for (int i = threadIdx.x; i < a.nd; i += kThreads) d += a.dpart[i];
#pragma unroll 4
    for (int i = threadIdx.x; i < a.ns; i += kThreads) s += a.spart[i];
#pragma unroll 4
    for (int i = threadIdx.x; i < a.ng; i += kThreads) {
        m = fmax(m, a.gpart[2 * i]);
        q += a.gpart[2 * i + 1];
    }
    d = rd_wave_sum(d);
    s = rd_wave_sum(s);
    m = rd_wave_max(m);
    q = rd_wave_sum(q);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[0][w] = d;
        sh[1][w] = s;
        sh[2][w] = m;
        sh[3][w] = q;
    }
    __syncthreads();
    d = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
    s = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
    const double gm = fmax(fmax(sh[2][0], sh[2][1]), fmax(sh[2][2], sh[2][3]));
    const double g2 = (sh[3][0] + sh[3][1]) + (sh[3][2] + sh[3][3]);
    if (threadIdx.x == 0) {
        const double D = a.half_hbar * d;
        const double S = a.half_hbary * s;
        const double J = D + a.alpha * S;
        a.out[0] = J;
        a.out[1] = D;
        a.out[2] = S;
        // fmax drops NaN, the sum of squares keeps it: a gradient with a NaN
        // or infinite entry reports a non-finite maximum, which ends L-BFGS
        // with the non-finite outcome
        a.out[3] = isfinite(g2) ? gm : g2;
        a.out[4] = g2;
        if (a.lb) lb_decide_one(a.lb, J);
    }
}

}  // namespace

}  // namespace ngf
