// Auxiliaries of the L-BFGS levels: the per-iteration log and checkpoint /
// resume of a level's state (Sec. 2.1: L-BFGS after Nocedal, 1980, whose
// state between two iterations is the iterate, its gradient and the stored
// correction pairs).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ngfreg.h"
#include "ngf_ctx.h"
#include "ngf_internal.h"

using namespace ngf;
using namespace ngf_host;

namespace {

// Tick of the level's start, before its first round.
__global__ void k_log_start(IterDev* rec) {
    if (threadIdx.x == 0 && blockIdx.x == 0) rec[0].tick = wall_clock64();
}

// After the evaluation of a round: when the round's trial was accepted (the
// reduction has taken the Armijo decision, the history update and the
// iteration count follow in the round's next kernels), record the step.
__global__ void k_log_round(const LbState* st, const double* jds, IterDev* rec, int cap) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const LbCtl& c = st->ctl;
    if (c.phase != kPhAccepted) return;
    const int k = c.iters + 1;
    if (k >= cap) return;
    IterDev r;
    r.iter = k;
    r.evals = c.evals;
    r.J = jds[0];
    r.D = jds[1];
    r.S = jds[2];
    r.gmax = jds[3];
    r.t = c.t;
    r.tick = wall_clock64();
    rec[k] = r;
}

ngf_status hip_fail(ngf_ctx* c, hipError_t e, const char* what) {
    (void)hipGetLastError();
    return fail(c, NGF_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

ngf_iter_record host_record(const ngf_ctx* c, int iter, double t, double us) {
    ngf_iter_record r{};
    r.level = c->lb_level;
    r.iter = iter;
    r.evals = c->lb_evals;
    r.J = c->host_jds[0];
    r.D = c->host_jds[1];
    r.S = c->host_jds[2];
    r.gmax = c->host_jds[3];
    r.t = t;
    r.us = us;
    return r;
}

// ---- checkpoint format -----------------------------------------------------

constexpr char kMagic[8] = {'N', 'G', 'F', 'L', 'B', 'F', 'G', 'S'};
constexpr uint32_t kVersion = 1;

struct StateHeader {
    char magic[8];
    uint32_t version;
    uint32_t state_bytes;  // sizeof(LbState) of the saving build
    int32_t level;
    int32_t my[3];
    int32_t mem;
    int32_t nslots;  // stored pairs that follow
    int64_t n;       // floats per vector (3 m^y)
    double J, gmax;
    int32_t evals, iters;
};
static_assert(sizeof(StateHeader) % 8 == 0, "header keeps the payload 8-byte aligned");

// stored pair: slot index (padded to 8 bytes), then s and t
size_t pair_bytes(int64_t n) { return 8 + 2 * static_cast<size_t>(n) * sizeof(float); }

size_t state_bytes(int64_t n, int nslots) {
    size_t b = sizeof(StateHeader) + sizeof(LbState);
    b = (b + 7) & ~size_t{7};
    return b + 2 * static_cast<size_t>(n) * sizeof(float) + nslots * pair_bytes(n);
}

size_t payload_offset() { return (sizeof(StateHeader) + sizeof(LbState) + 7) & ~size_t{7}; }

// Device state block of the running level, read back (synchronises).
ngf_status read_state(const ngf_ctx* c, LbState* out) {
    hipError_t e = hipMemcpyAsync(out, c->st, sizeof(LbState), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return NGF_E_HIP;
    }
    return NGF_OK;
}

}  // namespace

namespace ngf_host {

void log_start_point(ngf_ctx* c) {
    if (!c->log_on) return;
    c->log.push_back(host_record(c, 0, 0.0, 0.0));
    c->log_prev = std::chrono::steady_clock::now();
}

void log_host_step(ngf_ctx* c, double t) {
    if (!c->log_on) return;
    const auto now = std::chrono::steady_clock::now();
    const double us = std::chrono::duration<double, std::micro>(now - c->log_prev).count();
    c->log_prev = now;
    c->log.push_back(host_record(c, c->lb_iters, t, us));
}

ngf_status log_level_begin(ngf_ctx* c) {
    const int need = c->p.max_iter + 1;
    if (c->log_dev_cap < need) {
        hipError_t e = hipStreamSynchronize(c->stream);  // queued rounds may use the old buffer
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
        if (c->log_dev) (void)hipFree(c->log_dev);
        c->log_dev = nullptr;
        c->log_dev_cap = 0;
        if (c->faults & NGF_FAULT_ALLOC)
            return fail(c, NGF_E_OOM, "hipMalloc failed: allocation failure injected");
        e = hipMalloc(reinterpret_cast<void**>(&c->log_dev), need * sizeof(IterDev));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            c->log_dev = nullptr;
            return fail(c, NGF_E_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
        }
        c->log_dev_cap = need;
    }
    hipLaunchKernelGGL(k_log_start, dim3(1), dim3(64), 0, c->stream, c->log_dev);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? NGF_OK : hip_fail(c, e, "k_log_start");
}

ngf_status log_round(ngf_ctx* c) {
    hipLaunchKernelGGL(k_log_round, dim3(1), dim3(64), 0, c->stream, c->st, c->jds, c->log_dev,
                       c->log_dev_cap);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? NGF_OK : hip_fail(c, e, "k_log_round");
}

ngf_status log_level_end(ngf_ctx* c, int iters) {
    if (iters <= 0) return NGF_OK;
    const int n = std::min(iters + 1, c->log_dev_cap);
    std::vector<IterDev> rec(n);
    hipError_t e = hipMemcpyAsync(rec.data(), c->log_dev, n * sizeof(IterDev),
                                  hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "iteration log read-back");
    int dev = 0, khz = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return hip_fail(c, e, "device wall-clock rate");
    const double us_per_tick = khz > 0 ? 1e3 / khz : 0.0;
    for (int k = 1; k < n; ++k) {
        ngf_iter_record r{};
        r.level = c->lb_level;
        r.iter = rec[k].iter;
        r.evals = rec[k].evals;
        r.J = rec[k].J;
        r.D = rec[k].D;
        r.S = rec[k].S;
        r.gmax = rec[k].gmax;
        r.t = rec[k].t;
        r.us = static_cast<double>(rec[k].tick - rec[k - 1].tick) * us_per_tick;
        c->log.push_back(r);
    }
    return NGF_OK;
}

void log_free(ngf_ctx* c) {
    if (c->log_dev) (void)hipFree(c->log_dev);
    c->log_dev = nullptr;
    c->log_dev_cap = 0;
}

}  // namespace ngf_host

extern "C" {

ngf_status ngf_set_iteration_log(ngf_ctx* c, int32_t enable) {
    if (!c) return NGF_E_ARG;
    c->log_on = enable != 0;
    c->log.clear();
    return NGF_OK;
}

ngf_status ngf_iteration_log(const ngf_ctx* c, ngf_iter_record* out, int32_t cap,
                             int32_t* count) {
    if (!c || !count || cap < 0 || (cap > 0 && !out)) return NGF_E_ARG;
    const size_t n = std::min(c->log.size(), static_cast<size_t>(cap));
    if (n) std::memcpy(out, c->log.data(), n * sizeof(ngf_iter_record));
    *count = static_cast<int32_t>(c->log.size());
    return NGF_OK;
}

ngf_status ngf_lbfgs_state_size(const ngf_ctx* c, size_t* bytes) {
    if (!c || !bytes) return NGF_E_ARG;
    if (c->lb_level < 0 || c->lb_level >= static_cast<int>(c->lv.size())) return NGF_E_STATE;
    LbState st;
    const ngf_status s = read_state(c, &st);
    if (s != NGF_OK) return s;
    *bytes = state_bytes(3 * c->lv[c->lb_level].Ny(), st.count);
    return NGF_OK;
}

ngf_status ngf_lbfgs_save(ngf_ctx* c, void* buf, size_t bytes) {
    if (!c) return NGF_E_ARG;
    if (c->lb_level < 0 || c->lb_level >= static_cast<int>(c->lv.size()))
        return fail(c, NGF_E_STATE, "ngf_lbfgs_reset first");
    if (!buf) return fail(c, NGF_E_ARG, "null buffer");
    const Level& L = c->lv[c->lb_level];
    const int64_t n = 3 * L.Ny();
    LbState st;
    if (read_state(c, &st) != NGF_OK) return fail(c, NGF_E_HIP, "state read-back failed");
    if (st.count < 0 || st.count > kSlots) return fail(c, NGF_E_STATE, "corrupt L-BFGS state");
    const size_t need = state_bytes(n, st.count);
    if (bytes < need) return fail(c, NGF_E_ARG, "buffer smaller than ngf_lbfgs_state_size");
    char* p = static_cast<char*>(buf);
    StateHeader h{};
    std::memcpy(h.magic, kMagic, sizeof(kMagic));
    h.version = kVersion;
    h.state_bytes = sizeof(LbState);
    h.level = c->lb_level;
    for (int d = 0; d < 3; ++d) h.my[d] = L.my[d];
    h.mem = c->p.lbfgs_mem;
    h.nslots = st.count;
    h.n = n;
    h.J = c->lb_J;
    h.gmax = c->lb_gmax;
    h.evals = c->lb_evals;
    h.iters = c->lb_iters;
    std::memcpy(p, &h, sizeof(h));
    std::memcpy(p + sizeof(h), &st, sizeof(st));
    char* q = p + payload_offset();
    const size_t vb = static_cast<size_t>(n) * sizeof(float);
    hipError_t e = hipMemcpyAsync(q, c->ly, vb, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(q + vb, c->lg, vb, hipMemcpyDeviceToHost, c->stream);
    q += 2 * vb;
    for (int k = 0; k < st.count && e == hipSuccess; ++k) {
        const int64_t slot = st.order[k];
        if (slot < 0 || slot >= kSlots) return fail(c, NGF_E_STATE, "corrupt L-BFGS state");
        std::memset(q, 0, 8);
        std::memcpy(q, &slot, sizeof(slot));
        const float* row = c->hist + 2 * slot * static_cast<int64_t>(c->lb_ld);
        e = hipMemcpyAsync(q + 8, row, vb, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(q + 8 + vb, row + c->lb_ld, vb, hipMemcpyDeviceToHost, c->stream);
        q += pair_bytes(n);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "state copy to the host");
    return NGF_OK;
}

ngf_status ngf_lbfgs_load(ngf_ctx* c, const void* buf, size_t bytes) {
    if (!c) return NGF_E_ARG;
    if (!buf) return fail(c, NGF_E_ARG, "null buffer");
    if (c->lv.empty()) return fail(c, NGF_E_STATE, "no pyramid");
    const char* p = static_cast<const char*>(buf);
    StateHeader h;
    if (bytes < sizeof(h) + sizeof(LbState)) return fail(c, NGF_E_ARG, "not an L-BFGS state");
    std::memcpy(&h, p, sizeof(h));
    if (std::memcmp(h.magic, kMagic, sizeof(kMagic)) != 0 || h.version != kVersion ||
        h.state_bytes != sizeof(LbState))
        return fail(c, NGF_E_ARG, "not an L-BFGS state of this library build");
    if (h.level < 0 || h.level >= static_cast<int>(c->lv.size()))
        return fail(c, NGF_E_LEVEL, "the saved level does not exist in this pyramid");
    const Level& L = c->lv[h.level];
    for (int d = 0; d < 3; ++d)
        if (h.my[d] != L.my[d]) return fail(c, NGF_E_SHAPE, "deformation grid differs");
    if (h.n != 3 * L.Ny()) return fail(c, NGF_E_SHAPE, "deformation grid differs");
    if (h.mem != c->p.lbfgs_mem) return fail(c, NGF_E_ARG, "L-BFGS memory differs");
    if (h.nslots < 0 || h.nslots > kSlots) return fail(c, NGF_E_ARG, "corrupt state");
    if (bytes != state_bytes(h.n, h.nslots)) return fail(c, NGF_E_ARG, "state size mismatch");
    LbState st;
    std::memcpy(&st, p + sizeof(h), sizeof(st));
    if (st.count != h.nslots) return fail(c, NGF_E_ARG, "corrupt state");
    st.reject_all = (c->faults & NGF_FAULT_REJECT_STEPS) ? 1 : 0;
    const int64_t n = h.n;
    const size_t vb = static_cast<size_t>(n) * sizeof(float);
    const char* q = p + payload_offset();
    hipError_t e = hipMemcpyAsync(c->st, &st, sizeof(st), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->ly, q, vb, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->lg, q + vb, vb, hipMemcpyHostToDevice, c->stream);
    q += 2 * vb;
    for (int k = 0; k < h.nslots && e == hipSuccess; ++k) {
        int64_t slot = -1;
        std::memcpy(&slot, q, sizeof(slot));
        if (slot < 0 || slot >= kSlots || slot != st.order[k]) {
            (void)hipStreamSynchronize(c->stream);
            return fail(c, NGF_E_ARG, "corrupt state");
        }
        float* row = c->hist + 2 * slot * static_cast<int64_t>(c->lb_ld);
        e = hipMemcpyAsync(row, q + 8, vb, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(row + c->lb_ld, q + 8 + vb, vb, hipMemcpyHostToDevice, c->stream);
        q += pair_bytes(n);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "state copy to the device");
    c->lb_level = h.level;
    c->lb_J = h.J;
    c->lb_gmax = h.gmax;
    c->lb_evals = h.evals;
    c->lb_iters = h.iters;
    return NGF_OK;
}

}  // extern "C"
