// L-BFGS on the device (Sec. 2.1: L-BFGS after Nocedal, 1980).
//
// The two-loop recursion d = -H g is run in coefficient space: every vector
// it forms is a linear combination of the basis {s_k, t_k (stored pairs), g},
// so with the float64 Gram matrix of that basis the recursion reduces to
// O(m^2) scalar work, and d is formed in one pass over the stored vectors.
// The Gram matrix is updated after each accepted step by one pass that forms
// the new pair and all its inner products.  In exact arithmetic this is the
// two-loop recursion; every inner product is accumulated in float64 and
// reduced in a fixed order.
//
// Storage: hist holds kSlots pairs, slot k at hist + 2 k ld (s) and
// hist + (2 k + 1) ld (t), with the row stride ld a multiple of 64 floats so
// that every row is 16-byte aligned for vector loads.  Basis index of s in slot k is k, of t in slot k is
// kSlots + k, of the gradient kBasisG.
#include "lb_bodies.h"

namespace ngf {

namespace {

__global__ void k_lb_init(LbState* st, int mem, double hmin, const double* jds, int max_iter,
                          int early_stop, double tol) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        lb_init_one(st, mem, hmin, jds, max_iter, early_stop, tol);
}

__global__ void k_lb_solve(LbState* st, double* jds) {
    __shared__ SolveLds w;
    lb_stage(st, w);
    if (threadIdx.x < 64) lb_solve_wave(st, jds, w);
}

__global__ __launch_bounds__(kThreads) void k_lb_combine(const LbState* st,
                                                         const float* __restrict__ hist,
                                                         int64_t ld, int64_t n,
                                                         const float* __restrict__ y,
                                                         const float* __restrict__ g,
                                                         float* __restrict__ d,
                                                         float* __restrict__ yt) {
    if (lb_streams(n))
        lb_combine_body<true>(st, hist, ld, n, y, g, d, yt, blockIdx.x, gridDim.x);
    else
        lb_combine_body<false>(st, hist, ld, n, y, g, d, yt, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(kThreads) void k_lb_axpy(const float* __restrict__ y,
                                                      const float* __restrict__ d, float t,
                                                      float* __restrict__ yt, int64_t n) {
    lb_axpy_body(y, d, t, yt, n, blockIdx.x, gridDim.x);
}

template <int CMAX>
__global__ __launch_bounds__(kThreads) void k_lb_update_dots(const LbState* st,
                                                             float* __restrict__ hist,
                                                             int64_t ld, int64_t n,
                                                             const float* __restrict__ y,
                                                             const float* __restrict__ yt,
                                                             const float* __restrict__ g,
                                                             const float* __restrict__ gt,
                                                             double* __restrict__ dotpart) {
    if (lb_streams(n))
        lb_update_dots_body<false, CMAX, true>(st, hist, ld, n, const_cast<float*>(y), yt,
                                               const_cast<float*>(g), gt, dotpart, blockIdx.x,
                                               gridDim.x);
    else
        lb_update_dots_body<false, CMAX, false>(st, hist, ld, n, const_cast<float*>(y), yt,
                                                const_cast<float*>(g), gt, dotpart, blockIdx.x,
                                                gridDim.x);
}

__global__ __launch_bounds__(kGramThreads) void k_lb_gram_update(LbState* st,
                                                                 const double* dotpart,
                                                                 int nblocks,
                                                                 const double* jds) {
    lb_gram_body(st, dotpart, nblocks, jds);
}

__global__ void k_lb_plan(LbState* st, double* jds) { lb_plan_body(st, jds); }

__global__ __launch_bounds__(kThreads) void k_lb_vec(const LbState* st,
                                                     const float* __restrict__ hist, int64_t ld,
                                                     int64_t n, const float* __restrict__ y,
                                                     const float* __restrict__ g,
                                                     float* __restrict__ d,
                                                     float* __restrict__ yt) {
    lb_vec_body(st, hist, ld, n, y, g, d, yt, blockIdx.x, gridDim.x, lb_streams(n));
}

template <int CMAX>
__global__ __launch_bounds__(kThreads) void k_lb_accept_dots(const LbState* st,
                                                             float* __restrict__ hist,
                                                             int64_t ld, int64_t n, float* y,
                                                             const float* __restrict__ yt,
                                                             float* g,
                                                             const float* __restrict__ gt,
                                                             double* __restrict__ dotpart) {
    if (st->ctl.phase != kPhAccepted) return;
    if (lb_streams(n))
        lb_update_dots_body<true, CMAX, true>(st, hist, ld, n, y, yt, g, gt, dotpart,
                                              blockIdx.x, gridDim.x);
    else
        lb_update_dots_body<true, CMAX, false>(st, hist, ld, n, y, yt, g, gt, dotpart,
                                               blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(kGramThreads) void k_lb_gram_plan(LbState* st,
                                                               const double* dotpart,
                                                               int nblocks, double* jds) {
    lb_gram_plan_body(st, dotpart, nblocks, jds);
}

// ---- batched forms: one launch over many pairs (see BlockRef) ------------

__global__ void k_lb_init_batch(const LbVecArgs* args) {
    const LbVecArgs& a = args[blockIdx.x];
    if (threadIdx.x == 0)
        lb_init_one(a.st, a.mem, a.hmin, a.jds, a.max_iter, a.early_stop, a.tol);
}

__global__ void k_lb_plan_batch(const LbVecArgs* args) {
    const LbVecArgs& a = args[blockIdx.x];
    lb_plan_body(a.st, a.jds);
}

__global__ __launch_bounds__(kThreads) void k_lb_vec_batch(const LbVecArgs* args,
                                                           const BlockRef* blk) {
    const BlockRef e = blk[blockIdx.x];
    if (e.pair < 0) return;
    const LbVecArgs& a = args[e.pair];
    lb_vec_body(a.st, a.hist, a.ld, a.n, a.y, a.g, a.d, a.yt, e.block, a.nblocks,
                lb_streams(a.n));
}

template <int CMAX>
__global__ __launch_bounds__(kThreads) void k_lb_accept_dots_batch(const LbVecArgs* args,
                                                                   const BlockRef* blk) {
    const BlockRef e = blk[blockIdx.x];
    if (e.pair < 0) return;
    const LbVecArgs& a = args[e.pair];
    if (a.st->ctl.phase != kPhAccepted) return;
    if (lb_streams(a.n))
        lb_update_dots_body<true, CMAX, true>(a.st, a.hist, a.ld, a.n, a.y, a.yt, a.g, a.gt,
                                              a.dotpart, e.block, a.nblocks);
    else
        lb_update_dots_body<true, CMAX, false>(a.st, a.hist, a.ld, a.n, a.y, a.yt, a.g, a.gt,
                                               a.dotpart, e.block, a.nblocks);
}

__global__ __launch_bounds__(kGramThreads) void k_lb_gram_plan_batch(const LbVecArgs* args) {
    const LbVecArgs& a = args[blockIdx.x];
    lb_gram_plan_body(a.st, a.dotpart, a.nblocks, a.jds);
}

__global__ void k_ctl_gather(const LbVecArgs* args, LbCtl* out, int npairs) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < npairs) out[p] = args[p].st->ctl;
}

}  // namespace

void launch_lb_plan(LbState* st, double* jds, hipStream_t s) {
    hipLaunchKernelGGL(k_lb_plan, dim3(1), dim3(64), 0, s, st, jds);
}

void launch_lb_vec(LbState* st, const float* hist, int64_t ld, int64_t n, const float* y,
                   const float* g, float* d, float* yt, hipStream_t s) {
    hipLaunchKernelGGL(k_lb_vec, dim3(lb_dot_blocks(n)), dim3(kThreads), 0, s, st, hist, ld, n,
                       y, g, d, yt);
}

void launch_lb_accept(LbState* st, float* hist, int64_t ld, int64_t n, float* y,
                      const float* yt, float* g, const float* gt, double* dotpart,
                      int nblocks, double* jds, int mem, hipStream_t s) {
    if (mem <= 5)
        hipLaunchKernelGGL(k_lb_accept_dots<5>, dim3(nblocks), dim3(kThreads), 0, s, st, hist,
                           ld, n, y, yt, g, gt, dotpart);
    else
        hipLaunchKernelGGL(k_lb_accept_dots<kMaxMem>, dim3(nblocks), dim3(kThreads), 0, s, st,
                           hist, ld, n, y, yt, g, gt, dotpart);
    hipLaunchKernelGGL(k_lb_gram_plan, dim3(1), dim3(kGramThreads), 0, s, st, dotpart,
                       nblocks, jds);
}

void launch_lb_init_batch(const LbVecArgs* args, int npairs, hipStream_t s) {
    hipLaunchKernelGGL(k_lb_init_batch, dim3(npairs), dim3(64), 0, s, args);
}

void launch_lb_plan_batch(const LbVecArgs* args, int npairs, hipStream_t s) {
    hipLaunchKernelGGL(k_lb_plan_batch, dim3(npairs), dim3(64), 0, s, args);
}

void launch_lb_vec_batch(const LbVecArgs* args, const BlockRef* blk, int nblk, hipStream_t s) {
    if (nblk > 0)
        hipLaunchKernelGGL(k_lb_vec_batch, dim3(nblk), dim3(kThreads), 0, s, args, blk);
}

void launch_lb_accept_batch(const LbVecArgs* args, const BlockRef* blk, int nblk, int npairs,
                            int mem, hipStream_t s) {
    if (nblk > 0) {
        if (mem <= 5)
            hipLaunchKernelGGL(k_lb_accept_dots_batch<5>, dim3(nblk), dim3(kThreads), 0, s, args,
                               blk);
        else
            hipLaunchKernelGGL(k_lb_accept_dots_batch<kMaxMem>, dim3(nblk), dim3(kThreads), 0, s,
                               args, blk);
    }
    hipLaunchKernelGGL(k_lb_gram_plan_batch, dim3(npairs), dim3(kGramThreads), 0, s, args);
}

void launch_ctl_gather(const LbVecArgs* args, LbCtl* out, int npairs, hipStream_t s) {
    hipLaunchKernelGGL(k_ctl_gather, dim3((npairs + 63) / 64), dim3(64), 0, s, args, out, npairs);
}

// Workgroups of the L-BFGS vector passes over n floats: a thread takes four
// consecutive floats per step, so one workgroup per kThreads such groups, at
// most kLbBlocks (then the passes stride over the vector).  The last n mod 4
// floats go to the first threads of workgroup 0.
int lb_dot_blocks(int64_t n) {
    int64_t b = ((n >> 2) + kThreads - 1) / kThreads;
    if (b > kLbBlocks) b = kLbBlocks;
    if (b < 1) b = 1;
    return static_cast<int>(b);
}

void launch_lb_init(LbState* st, int mem, double hmin, const double* jds, int max_iter,
                    int early_stop, double tol, hipStream_t s) {
    hipLaunchKernelGGL(k_lb_init, dim3(1), dim3(64), 0, s, st, mem, hmin, jds, max_iter,
                       early_stop, tol);
}

void launch_lb_solve(LbState* st, double* jds, hipStream_t s) {
    hipLaunchKernelGGL(k_lb_solve, dim3(1), dim3(64), 0, s, st, jds);
}

void launch_lb_combine(LbState* st, const float* hist, int64_t ld, int64_t n, const float* y,
                       const float* g, float* d, float* yt, hipStream_t s) {
    hipLaunchKernelGGL(k_lb_combine, dim3(lb_dot_blocks(n)), dim3(kThreads), 0, s, st, hist, ld,
                       n, y, g, d, yt);
}

void launch_lb_axpy(const float* y, const float* d, float t, float* yt, int64_t n,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_lb_axpy, dim3(lb_dot_blocks(n)), dim3(kThreads), 0, s, y, d, t, yt, n);
}

void launch_lb_update_dots(LbState* st, float* hist, int64_t ld, int64_t n, const float* y,
                           const float* yt, const float* g, const float* gt, double* dotpart,
                           int nblocks, int mem, hipStream_t s) {
    if (mem <= 5)
        hipLaunchKernelGGL(k_lb_update_dots<5>, dim3(nblocks), dim3(kThreads), 0, s, st, hist,
                           ld, n, y, yt, g, gt, dotpart);
    else
        hipLaunchKernelGGL(k_lb_update_dots<kMaxMem>, dim3(nblocks), dim3(kThreads), 0, s, st,
                           hist, ld, n, y, yt, g, gt, dotpart);
}

void launch_lb_gram_update(LbState* st, const double* dotpart, int nblocks, const double* jds,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_lb_gram_update, dim3(1), dim3(kGramThreads), 0, s, st, dotpart, nblocks,
                       jds);
}

}  // namespace ngf
