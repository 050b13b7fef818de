// Batched form: registration of many independent image pairs of different
// shapes (the method of Sec. 2, applied pair by pair) on one device.
//
// Graph mode (default).  Every pair has a context (pyramid, scratch, L-BFGS
// buffers) on the batch's stream.  The pairs go through the levels together:
// at each level one L-BFGS round of every pair is one fixed sequence of
// batched launches (vector update, image pass per variant group, node pass,
// reduction with the Armijo test, history update ending with the next
// round's plan, control-block gather), each covering all pairs through a
// block table.  The sequence is
// captured once per level as a hipGraph and replayed; the host reads the
// gathered control blocks between batches of replays and stops when every
// pair's level has ended.  The kernels run the single-pair bodies with each
// pair's own arguments, so a pair's result equals its single-pair
// registration with the same image-pass variants, bit for bit.  Variants are
// picked per level shape by the timed selection, with one table shared by
// all pairs of the batch.
//
// Thread mode.  A host scheduler hands pairs, largest first, to worker
// threads, each with its own context and stream; the device overlaps them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ngfreg.h"
#include "ngf_ctx.h"
#include "ngf_internal.h"

using namespace ngf;
using namespace ngf_host;

namespace {

struct Worker {
    hipStream_t stream = nullptr;
    ngf_ctx* ctx = nullptr;
};

}  // namespace

struct ngf_batch {
    ngf_params p{};
    int device = 0;
    int mode = 0;          // 0 graph, 1 worker threads
    int variant = -3;      // -3: the mode's default (graph: timed, threads: size rule)
    std::vector<Worker> workers;
    hipStream_t stream = nullptr;
    hipEvent_t start = nullptr;
    std::vector<ngf_ctx*> pctx;  // graph mode: one context per pair slot
    std::vector<std::pair<std::string, int>> tune;  // shared timed-selection table
    // device tables of the current level (graph mode), grown on demand
    char* dtab = nullptr;
    size_t dtab_cap = 0;
    LbCtl* hctl = nullptr;  // pinned
    size_t hctl_cap = 0;
    double* hJ = nullptr;   // pinned, one J per pair (ngf_batch_eval)
    size_t hJ_cap = 0;
    int nbuilt = 0;         // pairs whose pyramids the pair contexts hold
    std::string err;
};

namespace {

ngf_status bfail(ngf_batch* b, ngf_status s, const std::string& m) {
    b->err = m;
    return s;
}

int graph_variant(const ngf_batch* b) { return b->variant == -3 ? -1 : b->variant; }
int thread_variant(const ngf_batch* b) { return b->variant == -3 ? kVariantBySize : b->variant; }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Append the blocks of one pair to a block table, its range starting at a
// multiple of 8 (padding entries have pair = -1).
void add_blocks(std::vector<BlockRef>& t, int pair, int64_t nblocks) {
    while (t.size() % 8) t.push_back(BlockRef{-1, 0});
    for (int64_t k = 0; k < nblocks; ++k) t.push_back(BlockRef{pair, static_cast<int>(k)});
}

struct LevelTables {
    std::vector<ImagePassArgs> img0, img1;  // reset evaluation / round evaluation
    std::vector<NodePassArgs> node0, node1;
    std::vector<ReduceArgs> red0, red1;
    std::vector<LbVecArgs> vec;
    struct Group {
        int variant;
        bool pow2;
        std::vector<BlockRef> blk;
        size_t off = 0;
    };
    std::vector<Group> groups;
    std::vector<BlockRef> node_blk, vec_blk;
};

template <class T>
size_t put(std::vector<char>& host, const std::vector<T>& v) {
    const size_t off = align_up(host.size(), 256);
    host.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(host.data() + off, v.data(), v.size() * sizeof(T));
    return off;
}

// Pair contexts (one per pair slot, on the batch stream) holding the
// pyramids of the pairs.
ngf_status build_pairs(ngf_batch* b, int np, const float* const* R, const float* const* T,
                       const ngf_grid* grids) {
    b->nbuilt = 0;
    while (static_cast<int>(b->pctx.size()) < np) {
        ngf_ctx* c = nullptr;
        const ngf_status s = ngf_create(&b->p, b->stream, &c);
        if (s != NGF_OK) return bfail(b, s, "ngf_create failed for a pair context");
        b->pctx.push_back(c);
    }
    const int var = graph_variant(b);
    for (int i = 0; i < np; ++i) {
        ngf_ctx* c = b->pctx[i];
        c->p = b->p;
        if (ngf_set_kernel(c, var) != NGF_OK) return bfail(b, NGF_E_ARG, c->err);
        // the shared timed-selection table: in before the pyramid, out after
        c->tune_loaded = true;
        c->tune_cache = b->tune;
        const ngf_status s = ngf_build_pyramid(c, R[i], T[i], &grids[i], 0);
        if (s != NGF_OK) return bfail(b, s, "pair " + std::to_string(i) + ": " + c->err);
        b->tune = c->tune_cache;
    }
    b->nbuilt = np;
    return NGF_OK;
}

// Upload a table image to the batch's device buffer (grown on demand, after
// the work queued on the batch stream is done).
ngf_status upload_tables(ngf_batch* b, const std::vector<char>& host, size_t bytes) {
    if (host.size() > b->dtab_cap) {
        if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, NGF_E_HIP, "sync");
        if (b->dtab) (void)hipFree(b->dtab);
        b->dtab = nullptr;
        b->dtab_cap = 0;
        if (hipMalloc(reinterpret_cast<void**>(&b->dtab), host.size() * 2) != hipSuccess)
            return bfail(b, NGF_E_OOM, "batch tables");
        b->dtab_cap = host.size() * 2;
    }
    if (hipMemcpyAsync(b->dtab, host.data(), bytes, hipMemcpyHostToDevice, b->stream) !=
            hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
        return bfail(b, NGF_E_HIP, "upload of the batch tables failed");
    return NGF_OK;
}

// One image pass per variant group, each covering its pairs' blocks.
void launch_image_groups(const std::vector<LevelTables::Group>& groups, const char* d,
                         size_t o_args, int ratio, hipStream_t s) {
    for (const auto& g : groups) {
        const auto* args = reinterpret_cast<const ImagePassArgs*>(d + o_args);
        const auto* blk = reinterpret_cast<const BlockRef*>(d + g.off);
        const int nb = static_cast<int>(g.blk.size());
        if (is_gen(g.variant))
            launch_image_gen_batch(args, blk, nb, g.pow2, s);
        else if (is_march(g.variant))
            launch_image_march_batch(args, blk, nb, ratio, g.variant, g.pow2, s);
        else
            launch_image_pass_batch(args, blk, nb, ratio, g.variant, g.pow2, s);
    }
}

// The variant group of a level in a block-table set.
LevelTables::Group& group_of(LevelTables& t, const Level& lv) {
    const bool p2 = pow2(lv.h[0]) && pow2(lv.h[1]) && pow2(lv.h[2]);
    for (auto& gg : t.groups)
        if (gg.variant == lv.variant && gg.pow2 == p2) return gg;
    t.groups.push_back(LevelTables::Group{lv.variant, p2, {}, 0});
    return t.groups.back();
}

ngf_status graph_register(ngf_batch* b, int np, const float* const* R, const float* const* T,
                          const ngf_grid* grids, float* const* y_out, ngf_report* reports) {
    if (const ngf_status s = build_pairs(b, np, R, T, grids); s != NGF_OK) return s;
    if (reports)
        for (int i = 0; i < np; ++i) {
            std::memset(&reports[i], 0, sizeof(ngf_report));
            reports[i].levels = b->p.levels;
        }
    if (b->hctl_cap < static_cast<size_t>(np)) {
        if (b->hctl) (void)hipHostFree(b->hctl);
        b->hctl = nullptr;
        b->hctl_cap = 0;
        if (hipHostMalloc(reinterpret_cast<void**>(&b->hctl), np * sizeof(LbCtl),
                          hipHostMallocDefault) != hipSuccess)
            return bfail(b, NGF_E_OOM, "pinned control-block buffer");
        b->hctl_cap = np;
    }
    hipStream_t s = b->stream;
    const int L = b->p.levels;
    for (int lev = L - 1; lev >= 0; --lev) {
        const auto t_level = std::chrono::steady_clock::now();
        LevelTables t;
        int max_iter = b->p.max_iter;
        for (int i = 0; i < np; ++i) {
            ngf_ctx* c = b->pctx[i];
            const Level& lv = c->lv[lev];
            // start point: identity on the coarsest level, else the prolongated
            // result of the coarser level
            if (lev == L - 1) {
                launch_identity(c->ltmp, lv.my[0], lv.my[1], lv.my[2], lv.hy[0], lv.hy[1],
                                lv.hy[2], s);
            } else {
                const Level& C = c->lv[lev + 1];
                launch_prolongate(c->ly, c->ltmp, C.my[0], C.my[1], C.my[2], s);
            }
            const int64_t n = 3 * lv.Ny();
            if (hipMemcpyAsync(c->ly, c->ltmp, n * sizeof(float), hipMemcpyDeviceToDevice, s) !=
                hipSuccess)
                return bfail(b, NGF_E_HIP, "hipMemcpyAsync of a start point failed");
            c->lb_level = lev;
            const EvalArgs e0 = eval_args(c, lv, lv.R, lv.T, c->ly, c->lg, nullptr, nullptr);
            const EvalArgs e1 =
                eval_args(c, lv, lv.R, lv.T, c->lyt, c->lgt, &c->st->ctl.op, c->st);
            t.img0.push_back(e0.a);
            t.img1.push_back(e1.a);
            t.node0.push_back(e0.b);
            t.node1.push_back(e1.b);
            t.red0.push_back(e0.r);
            t.red1.push_back(e1.r);
            LbVecArgs v{};
            v.st = c->st;
            v.hist = c->hist;
            v.ld = static_cast<int64_t>(c->lb_ld);
            v.n = n;
            v.y = c->ly;
            v.g = c->lg;
            v.d = c->ld;
            v.yt = c->lyt;
            v.gt = c->lgt;
            v.dotpart = c->dotpart;
            v.nblocks = lb_dot_blocks(n);
            v.jds = c->jds;
            v.mem = b->p.lbfgs_mem;
            v.max_iter = b->p.max_iter;
            v.early_stop = b->p.early_stop;
            v.hmin = std::min(lv.h[0], std::min(lv.h[1], lv.h[2]));
            v.tol = b->p.tol_J;
            t.vec.push_back(v);
            // block tables
            add_blocks(group_of(t, lv).blk, i, geometry(lv, lv.variant).ntiles());
            add_blocks(t.node_blk, i, node_blocks(lv));
            add_blocks(t.vec_blk, i, v.nblocks);
        }
        // upload the tables (one device buffer, grown outside the rounds)
        std::vector<char> host;
        const size_t o_img0 = put(host, t.img0), o_img1 = put(host, t.img1);
        const size_t o_node0 = put(host, t.node0), o_node1 = put(host, t.node1);
        const size_t o_red0 = put(host, t.red0), o_red1 = put(host, t.red1);
        const size_t o_vec = put(host, t.vec);
        for (auto& g : t.groups) g.off = put(host, g.blk);
        const size_t o_nblk = put(host, t.node_blk);
        const size_t o_vblk = put(host, t.vec_blk);
        const size_t o_ctl = align_up(host.size(), 256);
        host.resize(o_ctl + np * sizeof(LbCtl));
        // the previous level's graph has finished reading the tables (the
        // control blocks were read back after its last replay)
        if (const ngf_status us = upload_tables(b, host, o_ctl); us != NGF_OK) return us;
        char* d = b->dtab;
        auto P = [&](size_t off) { return static_cast<void*>(d + off); };
        const int ratio = b->p.ratio;
        auto image_stage = [&](size_t o_args) { launch_image_groups(t.groups, d, o_args, ratio, s); };
        const auto* vec = static_cast<const LbVecArgs*>(P(o_vec));
        const int nvb = static_cast<int>(t.vec_blk.size());
        auto node_stage = [&](size_t o_args) {
            launch_node_pass_batch(static_cast<const NodePassArgs*>(P(o_args)),
                                   static_cast<const BlockRef*>(P(o_nblk)),
                                   static_cast<int>(t.node_blk.size()), s);
        };
        // level start: evaluation at the start point, state reset
        image_stage(o_img0);
        node_stage(o_node0);
        launch_reduce_batch(static_cast<const ReduceArgs*>(P(o_red0)), np, s);
        launch_lb_init_batch(vec, np, s);
        launch_lb_plan_batch(vec, np, s);  // later plans end the rounds before them
        if (hipGetLastError() != hipSuccess) return bfail(b, NGF_E_HIP, "level start launch");
        // one round of every pair, captured once
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess)
            return bfail(b, NGF_E_HIP, "hipStreamBeginCapture failed");
        launch_lb_vec_batch(vec, static_cast<const BlockRef*>(P(o_vblk)), nvb, s);
        image_stage(o_img1);
        node_stage(o_node1);
        launch_reduce_batch(static_cast<const ReduceArgs*>(P(o_red1)), np, s);
        launch_lb_accept_batch(vec, static_cast<const BlockRef*>(P(o_vblk)), nvb, np,
                               b->p.lbfgs_mem, s);
        launch_ctl_gather(vec, static_cast<LbCtl*>(P(o_ctl)), np, s);
        const hipError_t ec = hipStreamEndCapture(s, &graph);
        if (ec != hipSuccess || !graph)
            return bfail(b, NGF_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return bfail(b, NGF_E_HIP, "hipGraphInstantiate failed");
        }
        ngf_status st = NGF_OK;
        const int64_t cap = static_cast<int64_t>(max_iter) * 11 + 2;
        int64_t rounds = 0;
        int batch = std::max(1, std::min(kRoundBatch, max_iter));
        for (;;) {
            for (int k = 0; k < batch && st == NGF_OK; ++k)
                if (hipGraphLaunch(exec, s) != hipSuccess) st = bfail(b, NGF_E_HIP, "hipGraphLaunch");
            rounds += batch;
            if (st != NGF_OK) break;
            if (hipMemcpyAsync(b->hctl, P(o_ctl), np * sizeof(LbCtl), hipMemcpyDeviceToHost, s) !=
                    hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                st = bfail(b, NGF_E_HIP, "control-block read failed");
                break;
            }
            bool done = true;
            int left = 1;
            for (int i = 0; i < np; ++i) {
                done = done && b->hctl[i].phase == kPhDone;
                if (b->hctl[i].phase != kPhDone)
                    left = std::max(left, b->hctl[i].max_iter - b->hctl[i].iters);
            }
            if (done) break;
            if (rounds > cap) {
                st = bfail(b, NGF_E_STATE, "device line search did not terminate");
                break;
            }
            batch = std::max(1, std::min(kRoundBatch, left));
        }
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        if (st != NGF_OK) return st;
        const double ms = std::chrono::duration<double, std::milli>(
                              std::chrono::steady_clock::now() - t_level)
                              .count();
        for (int i = 0; i < np; ++i) {
            ngf_ctx* c = b->pctx[i];
            const LbCtl& h = b->hctl[i];
            c->lb_J = h.J;
            c->lb_gmax = h.gmax;
            c->lb_evals = h.evals;
            if (reports) {
                reports[i].iters[lev] = h.iters;
                reports[i].evals[lev] = h.evals;
                reports[i].J[lev] = h.J;
                reports[i].info[lev] = h.info;
                reports[i].ms[lev] = ms;
            }
        }
    }
    for (int i = 0; i < np; ++i) {
        ngf_ctx* c = b->pctx[i];
        const size_t n = static_cast<size_t>(3 * c->lv[0].Ny());
        if (hipMemcpyAsync(y_out[i], c->ly, n * sizeof(float), hipMemcpyDeviceToDevice, s) !=
            hipSuccess)
            return bfail(b, NGF_E_HIP, "copy of a result failed");
    }
    if (hipStreamSynchronize(s) != hipSuccess) return bfail(b, NGF_E_HIP, "final sync failed");
    return NGF_OK;
}

// J and grad J of every built pair at level `lev`: one image pass per
// variant group, one node pass and one reduction, each covering all pairs.
ngf_status batch_eval(ngf_batch* b, int lev, const float* const* y, double* J,
                      float* const* grad) {
    const int np = b->nbuilt;
    hipStream_t s = b->stream;
    LevelTables t;
    std::vector<ReduceArgs> red;
    for (int i = 0; i < np; ++i) {
        ngf_ctx* c = b->pctx[i];
        if (lev < 0 || lev >= static_cast<int>(c->lv.size()))
            return bfail(b, NGF_E_LEVEL, "level out of range");
        const Level& lv = c->lv[lev];
        // the batched kernels always form the gradient: for J alone it goes
        // to the pair context's trial-gradient vector (sized for level 0)
        float* gi = grad ? grad[i] : c->lgt;
        const EvalArgs e = eval_args(c, lv, lv.R, lv.T, y[i], gi, nullptr, nullptr);
        t.img0.push_back(e.a);
        t.node0.push_back(e.b);
        red.push_back(e.r);
        add_blocks(group_of(t, lv).blk, i, geometry(lv, lv.variant).ntiles());
        add_blocks(t.node_blk, i, node_blocks(lv));
    }
    std::vector<char> host;
    const size_t o_img = put(host, t.img0), o_node = put(host, t.node0), o_red = put(host, red);
    for (auto& g : t.groups) g.off = put(host, g.blk);
    const size_t o_nblk = put(host, t.node_blk);
    if (const ngf_status us = upload_tables(b, host, host.size()); us != NGF_OK) return us;
    const char* d = b->dtab;
    launch_image_groups(t.groups, d, o_img, b->p.ratio, s);
    launch_node_pass_batch(reinterpret_cast<const NodePassArgs*>(d + o_node),
                           reinterpret_cast<const BlockRef*>(d + o_nblk),
                           static_cast<int>(t.node_blk.size()), s);
    launch_reduce_batch(reinterpret_cast<const ReduceArgs*>(d + o_red), np, s);
    if (hipGetLastError() != hipSuccess) return bfail(b, NGF_E_HIP, "batched evaluation launch");
    if (J) {
        if (b->hJ_cap < static_cast<size_t>(np)) {
            if (b->hJ) (void)hipHostFree(b->hJ);
            b->hJ = nullptr;
            b->hJ_cap = 0;
            if (hipHostMalloc(reinterpret_cast<void**>(&b->hJ), np * sizeof(double),
                              hipHostMallocDefault) != hipSuccess)
                return bfail(b, NGF_E_OOM, "pinned J buffer");
            b->hJ_cap = np;
        }
        for (int i = 0; i < np; ++i)
            if (hipMemcpyAsync(b->hJ + i, b->pctx[i]->jds, sizeof(double), hipMemcpyDeviceToHost,
                               s) != hipSuccess)
                return bfail(b, NGF_E_HIP, "copy of J failed");
    }
    if (hipStreamSynchronize(s) != hipSuccess) return bfail(b, NGF_E_HIP, "evaluation failed");
    if (J)
        for (int i = 0; i < np; ++i) J[i] = b->hJ[i];
    return NGF_OK;
}

ngf_status thread_register(ngf_batch* b, int npairs, const float* const* R,
                           const float* const* T, const ngf_grid* grids, float* const* y_out,
                           ngf_report* reports) {
    for (Worker& k : b->workers)
        if (hipStreamWaitEvent(k.stream, b->start, 0) != hipSuccess)
            return bfail(b, NGF_E_HIP, "hipStreamWaitEvent failed");
    const int var = thread_variant(b);
    for (Worker& k : b->workers)
        if (ngf_set_kernel(k.ctx, var) != NGF_OK) return bfail(b, NGF_E_ARG, k.ctx->err);

    // longest processing time first: pairs by voxel count, descending
    std::vector<int> order(npairs);
    std::iota(order.begin(), order.end(), 0);
    auto voxels = [&](int i) {
        return static_cast<int64_t>(grids[i].m[0]) * grids[i].m[1] * grids[i].m[2];
    };
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return voxels(a) > voxels(c); });

    std::atomic<int> next{0};
    std::atomic<bool> stop{false};
    std::vector<ngf_status> status(npairs, NGF_OK);
    std::vector<std::string> msg(npairs);
    std::vector<int> done(npairs, 0);
    auto run = [&](Worker* k) {
        if (hipSetDevice(b->device) != hipSuccess) {
            stop = true;
            return;
        }
        for (;;) {
            if (stop.load()) return;
            const int q = next.fetch_add(1);
            if (q >= npairs) return;
            const int i = order[q];
            ngf_report rep{};
            const ngf_status s =
                ngf_register(k->ctx, R[i], T[i], &grids[i], y_out[i], 0, reports ? &rep : nullptr);
            status[i] = s;
            done[i] = 1;
            if (reports) reports[i] = rep;
            if (s != NGF_OK) {
                msg[i] = ngf_last_error(k->ctx);
                stop = true;
                return;
            }
        }
    };
    std::vector<std::thread> threads;
    threads.reserve(b->workers.size());
    for (Worker& k : b->workers) threads.emplace_back(run, &k);
    for (std::thread& t : threads) t.join();

    for (int i = 0; i < npairs; ++i)
        if (status[i] != NGF_OK) return bfail(b, status[i], "pair " + std::to_string(i) + ": " + msg[i]);
    for (int i = 0; i < npairs; ++i)
        if (!done[i]) return bfail(b, NGF_E_HIP, "a worker could not select the device");
    return NGF_OK;
}

}  // namespace

extern "C" {

ngf_status ngf_batch_create(const ngf_params* p, int32_t workers, ngf_batch** out) {
    if (!out || !p) return NGF_E_ARG;
    *out = nullptr;
    if (workers < 1 || workers > NGF_BATCH_MAX_WORKERS) return NGF_E_ARG;
    ngf_batch* b = new (std::nothrow) ngf_batch();
    if (!b) return NGF_E_OOM;
    b->p = *p;
    ngf_status s = NGF_OK;
    if (hipGetDevice(&b->device) != hipSuccess ||
        hipEventCreateWithFlags(&b->start, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
        s = NGF_E_HIP;
    for (int w = 0; w < workers && s == NGF_OK; ++w) {
        Worker k;
        if (hipStreamCreateWithFlags(&k.stream, hipStreamNonBlocking) != hipSuccess) {
            s = NGF_E_HIP;
            break;
        }
        s = ngf_create(p, k.stream, &k.ctx);
        b->workers.push_back(k);
    }
    if (s != NGF_OK) {
        ngf_batch_destroy(b);
        return s;
    }
    *out = b;
    return NGF_OK;
}

void ngf_batch_destroy(ngf_batch* b) {
    if (!b) return;
    for (Worker& k : b->workers) {
        if (k.ctx) ngf_destroy(k.ctx);
        if (k.stream) {
            (void)hipStreamSynchronize(k.stream);
            (void)hipStreamDestroy(k.stream);
        }
    }
    for (ngf_ctx* c : b->pctx) ngf_destroy(c);
    if (b->stream) {
        (void)hipStreamSynchronize(b->stream);
        (void)hipStreamDestroy(b->stream);
    }
    if (b->dtab) (void)hipFree(b->dtab);
    if (b->hctl) (void)hipHostFree(b->hctl);
    if (b->hJ) (void)hipHostFree(b->hJ);
    if (b->start) (void)hipEventDestroy(b->start);
    delete b;
}

const char* ngf_batch_last_error(const ngf_batch* b) {
    return b ? b->err.c_str() : "null batch";
}

ngf_status ngf_batch_set_kernel(ngf_batch* b, int32_t variant) {
    if (!b) return NGF_E_ARG;
    if (variant < kVariantBySize || variant >= kNumVariants)
        return bfail(b, NGF_E_ARG, "unknown variant");
    b->variant = variant;
    return NGF_OK;
}

ngf_status ngf_batch_set_mode(ngf_batch* b, int32_t mode) {
    if (!b) return NGF_E_ARG;
    if (mode != 0 && mode != 1) return bfail(b, NGF_E_ARG, "mode must be 0 or 1");
    b->mode = mode;
    return NGF_OK;
}

ngf_status ngf_batch_register(ngf_batch* b, int32_t npairs, const float* const* R,
                              const float* const* T, const ngf_grid* grids, float* const* y_out,
                              void* stream, ngf_report* reports) {
    if (!b) return NGF_E_ARG;
    if (npairs < 0) return bfail(b, NGF_E_ARG, "npairs must be >= 0");
    if (npairs == 0) return NGF_OK;
    if (!R || !T || !grids || !y_out) return bfail(b, NGF_E_ARG, "null array argument");
    for (int i = 0; i < npairs; ++i)
        if (!R[i] || !T[i] || !y_out[i])
            return bfail(b, NGF_E_ARG, "null pointer for pair " + std::to_string(i));
    // the inputs may still be written by work queued on the caller's stream
    if (hipEventRecord(b->start, static_cast<hipStream_t>(stream)) != hipSuccess)
        return bfail(b, NGF_E_HIP, "hipEventRecord on the caller's stream failed");
    if (b->mode == 1) {
        b->nbuilt = 0;  // the worker contexts do not keep the pairs
        return thread_register(b, npairs, R, T, grids, y_out, reports);
    }
    if (hipStreamWaitEvent(b->stream, b->start, 0) != hipSuccess)
        return bfail(b, NGF_E_HIP, "hipStreamWaitEvent failed");
    return graph_register(b, npairs, R, T, grids, y_out, reports);
}

ngf_status ngf_batch_build(ngf_batch* b, int32_t npairs, const float* const* R,
                           const float* const* T, const ngf_grid* grids, void* stream) {
    if (!b) return NGF_E_ARG;
    b->nbuilt = 0;
    if (npairs < 0) return bfail(b, NGF_E_ARG, "npairs must be >= 0");
    if (npairs == 0) return NGF_OK;
    if (!R || !T || !grids) return bfail(b, NGF_E_ARG, "null array argument");
    for (int i = 0; i < npairs; ++i)
        if (!R[i] || !T[i]) return bfail(b, NGF_E_ARG, "null pointer for pair " + std::to_string(i));
    if (hipEventRecord(b->start, static_cast<hipStream_t>(stream)) != hipSuccess ||
        hipStreamWaitEvent(b->stream, b->start, 0) != hipSuccess)
        return bfail(b, NGF_E_HIP, "ordering after the caller's stream failed");
    return build_pairs(b, npairs, R, T, grids);
}

ngf_status ngf_batch_eval(ngf_batch* b, int32_t level, const float* const* y, double* J,
                          float* const* grad, void* stream) {
    if (!b) return NGF_E_ARG;
    if (b->nbuilt == 0) return bfail(b, NGF_E_STATE, "no pairs built (ngf_batch_build)");
    if (!y) return bfail(b, NGF_E_ARG, "null y array");
    for (int i = 0; i < b->nbuilt; ++i)
        if (!y[i] || (grad && !grad[i]))
            return bfail(b, NGF_E_ARG, "null pointer for pair " + std::to_string(i));
    if (hipEventRecord(b->start, static_cast<hipStream_t>(stream)) != hipSuccess ||
        hipStreamWaitEvent(b->stream, b->start, 0) != hipSuccess)
        return bfail(b, NGF_E_HIP, "ordering after the caller's stream failed");
    return batch_eval(b, level, y, J, grad);
}

}  // extern "C"
