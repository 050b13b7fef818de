// Host-side state of a context (internal to the library): the pyramid, the
// evaluation scratch and the L-BFGS buffers, shared by the single-pair entry
// points and the batched driver.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <string>
#include <utility>
#include <vector>

#include "../../include/ngfreg.h"
#include "ngf_internal.h"

namespace ngf_host {

using namespace ngf;

struct Level {
    int m[3] = {0, 0, 0};
    int my[3] = {0, 0, 0};
    double h[3] = {0, 0, 0};
    double hy[3] = {0, 0, 0};
    float* R = nullptr;
    float* T = nullptr;
    int32_t* j0[3] = {nullptr, nullptr, nullptr};
    float* w0[3] = {nullptr, nullptr, nullptr};
    float* w1[3] = {nullptr, nullptr, nullptr};
    float4* rn = nullptr;   // reference side of the NGF term (general image pass)
    int variant = kTile3D;  // image-pass variant (autotuned or forced)
    // every axis has m^y = m/r + 1 for one r in {2, 4}: 2 or 4; otherwise 0
    // (then only the general image pass applies)
    int dyadic = 2;
    int64_t N() const { return static_cast<int64_t>(m[0]) * m[1] * m[2]; }
    int64_t Ny() const { return static_cast<int64_t>(my[0]) * my[1] * my[2]; }
};

struct LevelStore {
    int64_t cap_n = 0;               // floats in R and in T
    int cap_m[3] = {0, 0, 0};        // entries per index-map axis
    void* p[12] = {};                // R, T, then j0, w0, w1 per axis, then rn
};

constexpr int kProfMax = 4096;

// One accepted L-BFGS step as the device-driven search records it (slot k of
// the level's record buffer; slot 0 holds the tick of the level's start).
struct IterDev {
    int iter, evals;
    double J, D, S, gmax, t;
    unsigned long long tick;  // device wall clock
};

}  // namespace ngf_host

struct ngf_ctx {
    ngf_params p{};
    hipStream_t stream = nullptr;
    hipStream_t side[2] = {nullptr, nullptr};
    hipEvent_t join[3] = {nullptr, nullptr, nullptr};
    std::string err;
    std::vector<ngf_host::Level> lv;
    // device storage of the pyramid, per level, kept across pyramids and
    // reused whenever it is large enough for the new shape
    std::vector<ngf_host::LevelStore> store;

    // evaluation scratch (sized for level 0 by ngf_build_pyramid / ngf_reserve)
    float* part = nullptr;
    size_t part_cap = 0;  // floats
    double* dpart = nullptr;
    size_t dpart_cap = 0;
    double* spart = nullptr;
    double* gpart = nullptr;
    size_t nblk_cap = 0;
    double* jds = nullptr;       // device {J, D, S, max|g|, |g|^2, ...}
    double* host_jds = nullptr;  // pinned: 8 doubles, then room for an LbCtl
    int* dflag = nullptr;

    // L-BFGS
    size_t lb_cap = 0;  // floats per vector
    size_t lb_ld = 0;   // row stride of the history (multiple of 64 floats)
    float* ly = nullptr;
    float* lg = nullptr;
    float* lyt = nullptr;
    float* lgt = nullptr;
    float* ld = nullptr;
    float* ltmp = nullptr;
    float* hist = nullptr;
    ngf::LbState* st = nullptr;
    double* dotpart = nullptr;
    int lb_level = -1;
    double lb_J = 0.0;
    double lb_gmax = 0.0;
    int lb_evals = 0;
    int lb_iters = 0;  // accepted steps since ngf_lbfgs_reset

    // iteration log (ngf_set_iteration_log)
    bool log_on = false;
    std::vector<ngf_iter_record> log;
    ngf_host::IterDev* log_dev = nullptr;  // records of the running device-driven level
    int log_dev_cap = 0;
    std::chrono::steady_clock::time_point log_prev;  // host time of the last host record

    // float64 evaluation (precision study): one scratch buffer of doubles,
    // allocated on the first float64 evaluation and grown when a later one
    // needs more
    double* f64 = nullptr;
    size_t f64_cap = 0;  // doubles

    int faults = 0;            // failure injection (NGF_FAULT_*)
    bool host_driven = false;  // register_levels: host-side line search (one sync per trial)
    // level-0 deformation-grid nodes per axis set by ngf_set_node_grid (0: m/ratio + 1)
    int node_grid[3] = {0, 0, 0};

    // image-pass variant: -1 = autotune, else forced for every level
    int forced_variant = -1;  // also kVariantBySize
    bool tune_loaded = false;
    std::vector<std::pair<std::string, int>> tune_cache;  // shape key -> variant

    // differentiation form: grid and index maps of the last explicit pair
    ngf_host::Level pair;
    std::vector<void*> pair_owned;

    // profiling of the image-pass kernel
    bool prof = false;
    std::vector<hipEvent_t> ev;
    int nprof = 0;                 // records in use (events 2i, 2i + 1)
    std::vector<int> prof_level;   // pyramid level of each record (-1: explicit pair)
    int prof_only = -1;            // record this pyramid level only (-1: every launch)
};


namespace ngf_host {

// Tile geometry of an image-pass variant: image tile extent per axis.
struct Geo {
    int tx, ty, tz;
    int ntx, nty, ntz;
    int px, py, pz;  // nodes per tile block of the P^T partial sums
    int64_t ntiles() const { return static_cast<int64_t>(ntx) * nty * ntz; }
};
Geo geometry(const Level& L, int variant);
int tiles(int m, int t);
int64_t node_blocks(const Level& L);
int node_chunk(const Level& L);
ngf_status fail(ngf_ctx* c, ngf_status s, const std::string& msg);

// Arguments of the three kernels of one evaluation at level L of context c:
// y evaluated, gradient into grad (null: value only), results in c->jds;
// gate and decide as in ImagePassArgs / ReduceArgs.
struct EvalArgs {
    ImagePassArgs a;
    NodePassArgs b;
    ReduceArgs r;
};
EvalArgs eval_args(ngf_ctx* c, const Level& L, const float* R, const float* T, const float* y,
                   float* grad, const int* gate, LbState* decide);
bool pow2(double h);
void node_grid(const Level& L, int nb[3]);

// Partial-sum buffers of the differentiation form (null: the context's own).
struct ScatterBufs {
    double* dpart;
    double* spart;
    double* gpart;
};
ngf_status eval_scatter(ngf_ctx* c, const Level& P, const float* R, const float* T,
                        const float* y, const double* gscale, double* J, double* J_dev,
                        float* grad_y, float* grad_T, const ScatterBufs* sb);
// Device address of the static scratch array of the no-allocation entry
// point on the current device; taken once per device at context creation.
ngf_status static_scratch_setup(ngf_ctx* c);

// Iteration log hooks (no-ops while the log is off).
// After ngf_lbfgs_reset has read J at y0 into host_jds: the start record.
void log_start_point(ngf_ctx* c);
// After an accepted host-driven step of length t (host_jds holds the new point).
void log_host_step(ngf_ctx* c, double t);
// Device-driven level: before its first round (buffer, start tick), after
// the evaluation of every round (records an accepted step), and after the
// level has ended with `iters` accepted steps (copies the records back).
ngf_status log_level_begin(ngf_ctx* c);
ngf_status log_round(ngf_ctx* c);
ngf_status log_level_end(ngf_ctx* c, int iters);
void log_free(ngf_ctx* c);

}  // namespace ngf_host
