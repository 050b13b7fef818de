// Device body of the final reduction of an evaluation (J = D + alpha S of
// Eq. 1 from the block partials, max |grad J| and |grad J|^2), shared by the
// single-pair kernel and its batched form.
#pragma once

#include "ngf_internal.h"

namespace ngf {

namespace {

// Fixed-order sums of the per-block partials: thread t adds entries t,
// t + 256, ... in order, then a fixed tree over the 256 thread sums.
__device__ inline double block_sum_fixed(const double* a, int n, double* sh) {
    double s = 0.0;
#pragma unroll 4
    for (int i = threadIdx.x; i < n; i += kThreads) s += a[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ void reduce_body(const ReduceArgs& a) {
    __shared__ double sh[kThreads];
    const double d = block_sum_fixed(a.dpart, a.nd, sh);
    const double s = block_sum_fixed(a.spart, a.ns, sh);
    double gm = 0.0, g2 = 0.0;
    if (a.ng > 0) {
        double m = 0.0, q = 0.0;
#pragma unroll 4
        for (int i = threadIdx.x; i < a.ng; i += kThreads) {
            m = fmax(m, a.gpart[2 * i]);
            q += a.gpart[2 * i + 1];
        }
        sh[threadIdx.x] = m;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
            __syncthreads();
        }
        gm = sh[0];
        __syncthreads();
        sh[threadIdx.x] = q;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        g2 = sh[0];
    }
    if (threadIdx.x == 0) {
        const double D = a.half_hbar * d;
        const double S = a.half_hbary * s;
        const double J = D + a.alpha * S;
        a.out[0] = J;
        a.out[1] = D;
        a.out[2] = S;
        a.out[3] = gm;
        a.out[4] = g2;
        if (a.lb) lb_decide_one(a.lb, J);
    }
}

}  // namespace

}  // namespace ngf
