// Batched form: registration of many independent image pairs of different
// shapes (the method of Sec. 2, applied pair by pair).
//
// A host scheduler orders the pairs by voxel count, largest first, and hands
// them out through an atomic counter to worker threads (longest processing
// time first).  Every worker owns one context on its own non-blocking HIP
// stream and registers its pairs through the same entry point as a single
// registration, so each pair's result is the single-pair result of the same
// image-pass variant bit for bit.  The device runs the workers' streams
// concurrently: the fine levels of one pair fill the GPU while another
// pair's coarse levels, which are bound by launch latency and by the host
// round trip of the line search, overlap with them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ngfreg.h"
#include "ngf_internal.h"

namespace {

struct Worker {
    hipStream_t stream = nullptr;
    ngf_ctx* ctx = nullptr;
};

}  // namespace

struct ngf_batch {
    ngf_params p{};
    int device = 0;
    int variant = ngf::kVariantBySize;
    std::vector<Worker> workers;
    hipEvent_t start = nullptr;
    std::string err;
};

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
        hipEventCreateWithFlags(&b->start, hipEventDisableTiming) != hipSuccess)
        s = NGF_E_HIP;
    for (int w = 0; w < workers && s == NGF_OK; ++w) {
        Worker k;
        if (hipStreamCreateWithFlags(&k.stream, hipStreamNonBlocking) != hipSuccess) {
            s = NGF_E_HIP;
            break;
        }
        s = ngf_create(p, k.stream, &k.ctx);
        if (s == NGF_OK) s = ngf_set_kernel(k.ctx, b->variant);
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
    if (b->start) (void)hipEventDestroy(b->start);
    delete b;
}

const char* ngf_batch_last_error(const ngf_batch* b) {
    return b ? b->err.c_str() : "null batch";
}

ngf_status ngf_batch_set_kernel(ngf_batch* b, int32_t variant) {
    if (!b) return NGF_E_ARG;
    for (Worker& k : b->workers) {
        const ngf_status s = ngf_set_kernel(k.ctx, variant);
        if (s != NGF_OK) {
            b->err = ngf_last_error(k.ctx);
            return s;
        }
    }
    b->variant = variant;
    return NGF_OK;
}

ngf_status ngf_batch_register(ngf_batch* b, int32_t npairs, const float* const* R,
                              const float* const* T, const ngf_grid* grids, float* const* y_out,
                              void* stream, ngf_report* reports) {
    if (!b) return NGF_E_ARG;
    if (npairs < 0) {
        b->err = "npairs must be >= 0";
        return NGF_E_ARG;
    }
    if (npairs == 0) return NGF_OK;
    if (!R || !T || !grids || !y_out) {
        b->err = "null array argument";
        return NGF_E_ARG;
    }
    for (int i = 0; i < npairs; ++i)
        if (!R[i] || !T[i] || !y_out[i]) {
            b->err = "null pointer for pair " + std::to_string(i);
            return NGF_E_ARG;
        }
    // the inputs may still be written by work queued on the caller's stream
    if (hipEventRecord(b->start, static_cast<hipStream_t>(stream)) != hipSuccess) {
        b->err = "hipEventRecord on the caller's stream failed";
        return NGF_E_HIP;
    }
    for (Worker& k : b->workers)
        if (hipStreamWaitEvent(k.stream, b->start, 0) != hipSuccess) {
            b->err = "hipStreamWaitEvent failed";
            return NGF_E_HIP;
        }

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
        if (status[i] != NGF_OK) {
            b->err = "pair " + std::to_string(i) + ": " + msg[i];
            return status[i];
        }
    for (int i = 0; i < npairs; ++i)
        if (!done[i]) {
            b->err = "a worker could not select the device";
            return NGF_E_HIP;
        }
    return NGF_OK;
}

}  // extern "C"
