// Host side of the C ABI declared in include/ngfreg.h: context, pyramid,
// evaluation orchestration, L-BFGS driver and the multi-level registration.
// Every compute step runs in the HIP kernels of this library; this file only
// validates arguments, owns device buffers and enqueues work.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/ngfreg.h"
#include "ngf_ctx.h"
#include "ngf_internal.h"

using namespace ngf;
using namespace ngf_host;

namespace ngf_host {

ngf_status fail(ngf_ctx* c, ngf_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

// A named host-side range for tools that collect markers (rocprofv3
// --marker-trace); without such a tool the calls return at once.
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

#define HIPCHK(ctx, expr)                                                              \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(ctx, NGF_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <class T>
ngf_status dalloc(ngf_ctx* c, T** p, size_t count) {
    *p = nullptr;
    if (c && (c->faults & NGF_FAULT_ALLOC))
        return fail(c, NGF_E_OOM, "hipMalloc failed: allocation failure injected");
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, NGF_E_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    return NGF_OK;
}

void dfree(void* p) {
    if (p) (void)hipFree(p);
}

bool params_ok(const ngf_params* p, std::string* why) {
    if (!(std::isfinite(p->alpha) && p->alpha >= 0.0)) return *why = "alpha must be >= 0", false;
    if (!(std::isfinite(p->tau) && p->tau > 0.0)) return *why = "tau must be > 0", false;
    if (!(std::isfinite(p->rho) && p->rho > 0.0)) return *why = "rho must be > 0", false;
    if (p->levels < 1 || p->levels > NGF_MAX_LEVELS) return *why = "levels out of range", false;
    if (p->ratio != 2 && p->ratio != 4) return *why = "ratio must be 2 or 4", false;
    if (p->max_iter < 0) return *why = "max_iter must be >= 0", false;
    if (p->lbfgs_mem < 1 || p->lbfgs_mem > kMaxMem) return *why = "lbfgs_mem out of range", false;
    if (!(std::isfinite(p->tol_J) && p->tol_J >= 0.0)) return *why = "tol_J must be >= 0", false;
    return true;
}

int tiles(int m, int t) { return (m + t - 1) / t; }

// Nodes in the largest block of P^T partial sums over tiles of extent te
// along an axis: a tile's block runs from the lower node of its first image
// point to the upper node of its last.
// Image points in the largest index set of Eq. 3 along an axis (the points
// whose lower or upper node is j, over all nodes j).
int index_set_span(int m, int n) {
    int s = 0;
    for (int j = 0; j < n; ++j)
        s = std::max(s, first_at_least(j + 1, m, n) - first_at_least(j - 1, m, n));
    return s;
}

int block_nodes(int m, int n, int te) {
    int best = 0;
    for (int t0 = 0; t0 < m; t0 += te) {
        const int last = std::min(t0 + te, m) - 1;
        best = std::max(best, map_lower(last, m, n) + 2 - map_lower(t0, m, n));
    }
    return best;
}

Geo geometry(const Level& L, int variant) {
    Geo g{};
    if (is_gen(variant)) {
        g.ty = g.tz = 32;
        // the node pass adds the partial sums of at most two tiles per axis,
        // so every index set along x must meet at most two chunks: a chunk
        // of at least (span - 1) planes
        const int lo = std::max(4, (index_set_span(L.m[0], L.my[0]) + 2) / 4 * 4);
        g.tx = fit_chunk(L.m[0], int64_t{tiles(L.m[1], 32)} * tiles(L.m[2], 32), 4, lo,
                         image_gen_slots());
    } else if (is_tile3d(variant)) {
        g.tx = tile3d_x(variant);
        g.ty = tile3d_y(variant);
        g.tz = tile3d_z(variant);
    } else {
        g.ty = march_ty(variant);
        g.tz = march_tz(variant);
        g.tx = march_cx(variant);
        if (g.tx == 0)
            g.tx = fit_chunk(L.m[0], int64_t{tiles(L.m[1], g.ty)} * tiles(L.m[2], g.tz), 4, 4,
                             image_march_slots(g.ty, g.tz));
    }
    g.ntx = tiles(L.m[0], g.tx);
    g.nty = tiles(L.m[1], g.ty);
    g.ntz = tiles(L.m[2], g.tz);
    if (is_gen(variant)) {
        // this kernel takes the block extents as arguments: the nodes a
        // tile's points reach, at most
        g.px = block_nodes(L.m[0], L.my[0], g.tx);
        g.py = block_nodes(L.m[1], L.my[1], g.ty);
        g.pz = block_nodes(L.m[2], L.my[2], g.tz);
    } else {
        // the kernels for a ratio of 2 or 4 write blocks of tile/ratio + 1
        // nodes per axis, also where the level is narrower than the tile
        const int r = L.dyadic > 0 ? L.dyadic : 2;
        g.px = g.tx / r + 1;
        g.py = g.ty / r + 1;
        g.pz = g.tz / r + 1;
    }
    return g;
}
int64_t part_floats(const Level& L, int variant) {
    const Geo g = geometry(L, variant);
    return g.ntiles() * 3 * int64_t{g.px} * g.py * g.pz;
}
// whether an image-pass variant can run on a level
bool variant_ok(const Level& L, int v) { return !needs_dyadic(v) || L.dyadic != 0; }
bool pow2(double h) {
    int e = 0;
    return std::frexp(h, &e) == 0.5;
}
// node-pass x chunk (node planes), fitted like the image pass's
int node_chunk(const Level& L) {
    return fit_chunk(L.my[0], 3 * int64_t{tiles(L.my[1], kNMY)} * tiles(L.my[2], kNMZ), 1, 4,
                     node_march_slots(), kNodeChunkMax);
}
// node-pass workgroups per axis (one per node tile and component)
void node_grid(const Level& L, int nb[3]) {
    nb[0] = tiles(L.my[0], node_chunk(L));
    nb[1] = tiles(L.my[1], kNMY);
    nb[2] = tiles(L.my[2], kNMZ);
}
int64_t node_blocks(const Level& L) {
    int nb[3];
    node_grid(L, nb);
    return 3 * static_cast<int64_t>(nb[0]) * nb[1] * nb[2];
}

ngf_status ensure_scratch(ngf_ctx* c, const Level& L) {
    size_t pf = 0, nt = 0;
    for (int v = 0; v < kNumVariants; ++v) {
        if (!variant_ok(L, v)) continue;
        pf = std::max(pf, static_cast<size_t>(part_floats(L, v)));
        const Geo g = geometry(L, v);
        nt = std::max(nt, static_cast<size_t>(g.ntiles()));
        // the node pass addresses one x-slab of tile partials with 32-bit offsets
        const int64_t slab = int64_t{g.nty} * g.ntz * 3 * g.px * g.py * g.pz;
        if (slab >= (int64_t{1} << 31))
            return fail(c, NGF_E_SHAPE, "image too large in y and z for the tile layout");
    }
    const size_t nb = static_cast<size_t>(node_blocks(L));
    if (pf > c->part_cap || nt > c->dpart_cap || nb > c->nblk_cap)
        HIPCHK(c, hipStreamSynchronize(c->stream));  // queued work may use the old buffers
    if (pf > c->part_cap) {
        dfree(c->part);
        c->part = nullptr;
        c->part_cap = 0;
        if (dalloc(c, &c->part, pf) != NGF_OK) return NGF_E_OOM;
        c->part_cap = pf;
    }
    if (nt > c->dpart_cap) {
        dfree(c->dpart);
        c->dpart = nullptr;
        c->dpart_cap = 0;
        if (dalloc(c, &c->dpart, nt) != NGF_OK) return NGF_E_OOM;
        c->dpart_cap = nt;
    }
    if (nb > c->nblk_cap) {
        dfree(c->spart);
        dfree(c->gpart);
        c->spart = c->gpart = nullptr;
        c->nblk_cap = 0;
        if (dalloc(c, &c->spart, nb) != NGF_OK) return NGF_E_OOM;
        if (dalloc(c, &c->gpart, 2 * nb) != NGF_OK) return NGF_E_OOM;
        c->nblk_cap = nb;
    }
    return NGF_OK;
}

ngf_status ensure_lbfgs(ngf_ctx* c, size_t n) {
    if (n <= c->lb_cap) return NGF_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));  // queued work may use the old buffers
    for (float** p : {&c->ly, &c->lg, &c->lyt, &c->lgt, &c->ld, &c->ltmp, &c->hist}) {
        dfree(*p);
        *p = nullptr;
    }
    dfree(c->dotpart);
    c->dotpart = nullptr;
    c->lb_cap = 0;
    for (float** p : {&c->ly, &c->lg, &c->lyt, &c->lgt, &c->ld, &c->ltmp})
        if (dalloc(c, p, n) != NGF_OK) return NGF_E_OOM;
    c->lb_ld = (n + 63) / 64 * 64;
    if (dalloc(c, &c->hist, static_cast<size_t>(2) * kSlots * c->lb_ld) != NGF_OK)
        return NGF_E_OOM;
    if (dalloc(c, &c->dotpart, static_cast<size_t>(lb_dot_blocks(static_cast<int64_t>(n))) *
                                   (6 * kSlots + 6)) != NGF_OK)
        return NGF_E_OOM;
    c->lb_cap = n;
    return NGF_OK;
}

void free_pyramid(ngf_ctx* c) {
    for (LevelStore& st : c->store)
        for (void*& p : st.p) {
            dfree(p);
            p = nullptr;
        }
    c->store.clear();
    c->lv.clear();
}

// Point level l at storage of sufficient size, allocating only when the
// kept storage is too small (then after the context's queued work is done).
ngf_status bind_level_storage(ngf_ctx* c, int l) {
    Level& lv = c->lv[l];
    if (static_cast<int>(c->store.size()) <= l) c->store.resize(l + 1);
    LevelStore& st = c->store[l];
    bool fits = st.cap_n >= lv.N();
    for (int d = 0; d < 3; ++d) fits = fits && st.cap_m[d] >= lv.m[d];
    if (!fits) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (void*& p : st.p) {
            dfree(p);
            p = nullptr;
        }
        st.cap_n = 0;
        for (int d = 0; d < 3; ++d) st.cap_m[d] = 0;
        const size_t n = static_cast<size_t>(lv.N());
        // index maps are small: room for the longest axis (at least 1024)
        // on every axis, so that pairs of other shapes reuse them
        const int lng = std::max(1024, std::max(lv.m[0], std::max(lv.m[1], lv.m[2])));
        const int cap_m[3] = {lng, lng, lng};
        float* f = nullptr;
        if (dalloc(c, &f, n) != NGF_OK) return NGF_E_OOM;
        st.p[0] = f;
        if (dalloc(c, &f, n) != NGF_OK) return NGF_E_OOM;
        st.p[1] = f;
        float4* rn = nullptr;
        if (dalloc(c, &rn, n) != NGF_OK) return NGF_E_OOM;
        st.p[11] = rn;
        for (int d = 0; d < 3; ++d) {
            int32_t* j = nullptr;
            if (dalloc(c, &j, cap_m[d]) != NGF_OK) return NGF_E_OOM;
            st.p[2 + 3 * d] = j;
            for (int k = 1; k < 3; ++k) {
                if (dalloc(c, &f, cap_m[d]) != NGF_OK) return NGF_E_OOM;
                st.p[2 + 3 * d + k] = f;
            }
        }
        st.cap_n = lv.N();
        for (int d = 0; d < 3; ++d) st.cap_m[d] = cap_m[d];
    }
    lv.R = static_cast<float*>(st.p[0]);
    lv.T = static_cast<float*>(st.p[1]);
    lv.rn = static_cast<float4*>(st.p[11]);
    for (int d = 0; d < 3; ++d) {
        lv.j0[d] = static_cast<int32_t*>(st.p[2 + 3 * d]);
        lv.w0[d] = static_cast<float*>(st.p[3 + 3 * d]);
        lv.w1[d] = static_cast<float*>(st.p[4 + 3 * d]);
    }
    return NGF_OK;
}

ImagePassArgs image_args(ngf_ctx* c, const Level& L, const float* R, const float* T,
                         const float* y, bool grad) {
    ImagePassArgs a{};
    a.R = R;
    a.T = T;
    a.y = y;
    a.j0x = L.j0[0];
    a.j0y = L.j0[1];
    a.j0z = L.j0[2];
    a.w0x = L.w0[0];
    a.w0y = L.w0[1];
    a.w0z = L.w0[2];
    a.w1x = L.w1[0];
    a.w1y = L.w1[1];
    a.w1z = L.w1[2];
    a.rn = L.rn;
    a.part = c->part;
    a.dpart = c->dpart;
    a.mx = L.m[0];
    a.my = L.m[1];
    a.mz = L.m[2];
    a.nx = L.my[0];
    a.ny = L.my[1];
    a.nz = L.my[2];
    const Geo g = geometry(L, L.variant);
    a.ntx = g.ntx;
    a.nty = g.nty;
    a.ntz = g.ntz;
    a.cx = g.tx;
    a.px = g.px;
    a.py = g.py;
    a.pz = g.pz;
    a.hx = L.h[0];
    a.hy = L.h[1];
    a.hz = L.h[2];
    a.ihx = 1.0 / L.h[0];
    a.ihy = 1.0 / L.h[1];
    a.ihz = 1.0 / L.h[2];
    a.pow2h = pow2(L.h[0]) && pow2(L.h[1]) && pow2(L.h[2]);
    a.fihx = static_cast<float>(1.0 / L.h[0]);
    a.fihy = static_cast<float>(1.0 / L.h[1]);
    a.fihz = static_cast<float>(1.0 / L.h[2]);
    a.i2hx = static_cast<float>(0.5 / L.h[0]);
    a.i2hy = static_cast<float>(0.5 / L.h[1]);
    a.i2hz = static_cast<float>(0.5 / L.h[2]);
    a.tau = static_cast<float>(c->p.tau);
    a.rho = static_cast<float>(c->p.rho);
    a.hbar = static_cast<float>(L.h[0] * L.h[1] * L.h[2]);
    a.want_grad = grad ? 1 : 0;
    return a;
}

EvalArgs eval_args(ngf_ctx* c, const Level& L, const float* R, const float* T, const float* y,
                   float* grad, const int* gate, LbState* decide) {
    const bool want = grad != nullptr;
    EvalArgs e{};
    ImagePassArgs& a = e.a;
    a = image_args(c, L, R, T, y, want);
    a.gate = gate;
    NodePassArgs& b = e.b;
    b.y = y;
    b.part = c->part;
    b.grad = grad;
    b.spart = c->spart;
    b.gpart = c->gpart;
    b.nx = L.my[0];
    b.ny = L.my[1];
    b.nz = L.my[2];
    b.ntx = a.ntx;
    b.nty = a.nty;
    b.ntz = a.ntz;
    const Geo g = geometry(L, L.variant);
    b.tex = g.tx;
    b.tey = g.ty;
    b.tez = g.tz;
    b.mx = L.m[0];
    b.my = L.m[1];
    b.mz = L.m[2];
    b.px = g.px;
    b.py = g.py;
    b.pz = g.pz;
    int nb[3];
    node_grid(L, nb);
    b.nbx = nb[0];
    b.nby = nb[1];
    b.nbz = nb[2];
    b.cxn = node_chunk(L);
    b.hyx = L.hy[0];
    b.hyy = L.hy[1];
    b.hyz = L.hy[2];
    b.ihy2x = static_cast<float>(1.0 / (L.hy[0] * L.hy[0]));
    b.ihy2y = static_cast<float>(1.0 / (L.hy[1] * L.hy[1]));
    b.ihy2z = static_cast<float>(1.0 / (L.hy[2] * L.hy[2]));
    const double hbary = L.hy[0] * L.hy[1] * L.hy[2];
    b.alpha_hbary = static_cast<float>(c->p.alpha * hbary);
    b.alpha = static_cast<float>(c->p.alpha);
    b.want_grad = want ? 1 : 0;
    b.gather = 1;
    b.gscale = nullptr;
    b.gate = gate;
    ReduceArgs& r = e.r;
    r.dpart = c->dpart;
    r.nd = static_cast<int>(g.ntiles());
    r.spart = c->spart;
    r.ns = static_cast<int>(node_blocks(L));
    r.gpart = c->gpart;
    r.ng = want ? r.ns : 0;
    r.half_hbar = 0.5 * L.h[0] * L.h[1] * L.h[2];
    r.half_hbary = 0.5 * hbary;
    r.alpha = c->p.alpha;
    r.out = c->jds;
    r.gate = gate;
    r.lb = decide;
    return e;
}

// Enqueue one evaluation on the context stream; results land in c->jds and
// (if grad != nullptr) in grad.
ngf_status enqueue_eval(ngf_ctx* c, const Level& L, const float* R, const float* T,
                        const float* y, float* grad, const int* gate = nullptr,
                        LbState* decide = nullptr) {
    const EvalArgs e = eval_args(c, L, R, T, y, grad, gate, decide);
    auto launch = [&] {
        if (is_gen(L.variant))
            launch_image_gen(e.a, e.a.cx, c->stream);
        else if (!is_march(L.variant))
            launch_image_pass(e.a, L.dyadic, L.variant, c->stream);
        else
            launch_image_march(e.a, L.dyadic, march_ty(L.variant), march_tz(L.variant), e.a.cx,
                               c->stream);
    };
    int li = -1;
    if (c->prof)
        for (size_t l = 0; l < c->lv.size(); ++l)
            if (&c->lv[l] == &L) li = static_cast<int>(l);
    if (c->prof && c->nprof < kProfMax && (c->prof_only < 0 || li == c->prof_only)) {
        HIPCHK(c, hipEventRecord(c->ev[2 * c->nprof], c->stream));
        launch();
        HIPCHK(c, hipEventRecord(c->ev[2 * c->nprof + 1], c->stream));
        c->prof_level[c->nprof] = li;
        c->nprof++;
    } else {
        launch();
    }
    HIPCHK(c, hipGetLastError());
    launch_node_pass(e.b, c->stream);
    HIPCHK(c, hipGetLastError());
    launch_reduce(e.r, c->stream);
    HIPCHK(c, hipGetLastError());
    return NGF_OK;
}

ngf_status read_jds(ngf_ctx* c) {
    HIPCHK(c, hipMemcpyAsync(c->host_jds, c->jds, 8 * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return NGF_OK;
}

// Autotune cache key: the device's architecture name, the image grid and
// the deformation grid of a level.
std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');  // drop feature flags (gfx950:sramecc+:xnack-)
    if (colon != std::string::npos) a.resize(colon);
    return a.empty() ? "unknown" : a;
}
std::string tune_key(const Level& L) {
    char buf[160];
    std::snprintf(buf, sizeof(buf), "%s %d %d %d n%d,%d,%d", device_arch().c_str(), L.m[0],
                  L.m[1], L.m[2], L.my[0], L.my[1], L.my[2]);
    return buf;
}

void tune_cache_load(ngf_ctx* c) {
    const char* path = std::getenv("NGF_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char arch[64];
    int m0, m1, m2, n0, n1, n2, v;
    while (std::fscanf(f, "%63s %d %d %d n%d,%d,%d %d", arch, &m0, &m1, &m2, &n0, &n1, &n2,
                       &v) == 8) {
        if (v < 0 || v >= kNumVariants) continue;
        char buf[160];
        std::snprintf(buf, sizeof(buf), "%s %d %d %d n%d,%d,%d", arch, m0, m1, m2, n0, n1, n2);
        c->tune_cache.emplace_back(buf, v);
    }
    std::fclose(f);
}

void tune_cache_store(const std::string& key, int v) {
    const char* path = std::getenv("NGF_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d\n", key.c_str(), v);
    std::fclose(f);
}

// Image-pass variant from the level size alone, for callers that cannot
// afford timing runs (or whose timings would be disturbed by concurrent
// work): the fastest variants measured on gfx950 at cubic levels of 256^3
// and 128^3 (the 32 x 32 marching tile) and of 64^3 and below (the small 3D
// tile).
int variant_by_size(const Level& L) {
    if (!L.dyadic) return kMarchGen;
    return L.N() >= (int64_t{1} << 20) ? kMarchSqFit : kTile3DTiny;
}

// Pick the image-pass variant of every level: forced, cached for this shape,
// or the fastest of all variants over three timed evaluations at the identity
// (whole evaluation: image pass, node pass and reduction).
ngf_status autotune(ngf_ctx* c) {
    if (c->forced_variant >= 0) {
        // a variant that needs a ratio of 2 or 4 gives way to the general
        // pass on levels with other grids
        for (Level& L : c->lv)
            L.variant = variant_ok(L, c->forced_variant) ? c->forced_variant : kMarchGen;
        return NGF_OK;
    }
    if (c->forced_variant == kVariantBySize) {
        for (Level& L : c->lv) L.variant = variant_by_size(L);
        return NGF_OK;
    }
    if (!c->tune_loaded) {
        tune_cache_load(c);
        c->tune_loaded = true;
    }
    const bool prof = c->prof;
    c->prof = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    ngf_status st = NGF_OK;
    for (Level& L : c->lv) {
        const std::string key = tune_key(L);
        int found = -1;
        for (auto& kv : c->tune_cache)
            if (kv.first == key) found = kv.second;
        if (found >= 0) {
            L.variant = found;
            continue;
        }
        launch_identity(c->ltmp, L.my[0], L.my[1], L.my[2], L.hy[0], L.hy[1], L.hy[2],
                        c->stream);
        int best = L.dyadic ? kTile3D : kMarchGen;
        float best_ms = 1e30f;
        for (int v = 0; v < kNumVariants && st == NGF_OK; ++v) {
            if (!variant_ok(L, v)) continue;
            L.variant = v;
            st = enqueue_eval(c, L, L.R, L.T, c->ltmp, c->lgt);
            if (st != NGF_OK) break;
            if (hipEventRecord(e0, c->stream) != hipSuccess) st = NGF_E_HIP;
            for (int r = 0; r < 3 && st == NGF_OK; ++r)
                st = enqueue_eval(c, L, L.R, L.T, c->ltmp, c->lgt);
            if (st == NGF_OK && hipEventRecord(e1, c->stream) != hipSuccess) st = NGF_E_HIP;
            float ms = 0.0f;
            if (st == NGF_OK && (hipEventSynchronize(e1) != hipSuccess ||
                                 hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                st = fail(c, NGF_E_HIP, "autotune timing failed");
            if (st == NGF_OK && ms < best_ms) {
                best_ms = ms;
                best = v;
            }
        }
        L.variant = best;
        c->tune_cache.emplace_back(key, best);
        tune_cache_store(key, best);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->prof = prof;
    return st;
}

bool early_stop_met(double J_old, double J_new, double tol) {
#pragma clang fp contract(off)
    return (J_old - J_new) <= tol * (1.0 + std::fabs(J_old));
}

// Armijo test, rounded exactly as the device's (no contraction).
bool armijo_ok(double Jt, double J, double c1, double t, double gtd) {
#pragma clang fp contract(off)
    return std::isfinite(Jt) && Jt <= J + c1 * t * gtd;
}

// One round of the device-driven level: plan, vector update, gated
// evaluation of the trial point (its reduction also takes the Armijo
// decision), gated history update.
// Returns whether the round's image pass was recorded for profiling.
ngf_status enqueue_round(ngf_ctx* c, const Level& L, bool* recorded) {
    const int64_t n = 3 * L.Ny();
    const int* gate = &c->st->ctl.op;
    launch_lb_vec(c->st, c->hist, static_cast<int64_t>(c->lb_ld), n, c->ly, c->lg, c->ld,
                  c->lyt, c->stream);
    HIPCHK(c, hipGetLastError());
    const int before = c->nprof;
    const ngf_status e = enqueue_eval(c, L, L.R, L.T, c->lyt, c->lgt, gate, c->st);
    if (e != NGF_OK) return e;
    *recorded = c->nprof > before;
    if (c->log_on) {
        const ngf_status le = log_round(c);
        if (le != NGF_OK) return le;
    }
    launch_lb_accept(c->st, c->hist, static_cast<int64_t>(c->lb_ld), n, c->ly, c->lyt, c->lg,
                     c->lgt, c->dotpart, lb_dot_blocks(n), c->jds, c->p.lbfgs_mem, c->stream);
    HIPCHK(c, hipGetLastError());
    return NGF_OK;
}

// Run the L-BFGS iterations of the level set up by ngf_lbfgs_reset on the
// device: rounds are enqueued in batches and the control block is read back
// once per batch.  Rounds after the end of the level do nothing; their
// profiling records (if any) are dropped.  Same arithmetic and decisions as
// repeated ngf_lbfgs_step calls with the early-stop test between them.
ngf_status run_level_on_device(ngf_ctx* c, LbCtl* out) {
    const Level& L = c->lv[c->lb_level];
    const int64_t cap = static_cast<int64_t>(c->p.max_iter) * 11 + 2;  // rounds that can do work
    std::vector<char> rec;
    int64_t rounds = 0;
    // every round makes at most one step: size a batch by the remaining budget
    int batch = std::max(1, std::min(kRoundBatch, c->p.max_iter));
    LbCtl* h = reinterpret_cast<LbCtl*>(c->host_jds + 8);
    launch_lb_plan(c->st, c->jds, c->stream);  // later plans end the rounds before them
    HIPCHK(c, hipGetLastError());
    if (c->log_on) {
        const ngf_status le = log_level_begin(c);
        if (le != NGF_OK) return le;
    }
    for (;;) {
        for (int k = 0; k < batch; ++k) {
            bool r = false;
            const ngf_status e = enqueue_round(c, L, &r);
            if (e != NGF_OK) return e;
            rec.push_back(r ? 1 : 0);
            ++rounds;
        }
        HIPCHK(c, hipMemcpyAsync(h, &c->st->ctl, sizeof(LbCtl), hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (h->phase == kPhDone) break;
        if (rounds > cap) return fail(c, NGF_E_STATE, "device line search did not terminate");
        batch = std::max(1, std::min(kRoundBatch, h->max_iter - h->iters));
    }
    // rounds that ran an evaluation come first; drop the records of the rest
    const int64_t working = h->evals - 1;
    for (int64_t r = rounds - 1; r >= working && r >= 0; --r)
        if (rec[r]) c->nprof--;
    *out = *h;
    c->lb_J = h->J;
    c->lb_gmax = h->gmax;
    c->lb_evals = h->evals;
    c->lb_iters = h->iters;
    if (c->log_on) return log_level_end(c, h->iters);
    return NGF_OK;
}

ngf_status check_level(const ngf_ctx* c, int level) {
    if (c->lv.empty()) return NGF_E_STATE;
    if (level < 0 || level >= static_cast<int>(c->lv.size())) return NGF_E_LEVEL;
    return NGF_OK;
}


// J of the evaluation just queued: copied to J_dev (device) and read back to
// J (host, synchronises) when given.
ngf_status finish_J(ngf_ctx* c, double* J, double* J_dev) {
    if (J_dev)
        HIPCHK(c, hipMemcpyAsync(J_dev, c->jds, sizeof(double), hipMemcpyDeviceToDevice,
                                 c->stream));
    if (J) {
        if (read_jds(c) != NGF_OK) return NGF_E_HIP;
        *J = c->host_jds[0];
        if (!std::isfinite(*J)) return fail(c, NGF_E_NONFINITE, "J is not finite");
    }
    return NGF_OK;
}

// Differentiation form on level L (its grids and index maps) with images R, T:
// J, and grad_y / grad_T by atomic scatter (3D-tile kernel), alpha grad S
// added by the node pass.  Uses only buffers sized beforehand.
ngf_status eval_scatter(ngf_ctx* c, const Level& P, const float* R, const float* T,
                        const float* y, const double* gscale, double* J, double* J_dev,
                        float* grad_y, float* grad_T, const ScatterBufs* sb) {
    const int r = P.dyadic;
    double* dpart = sb ? sb->dpart : c->dpart;
    double* spart = sb ? sb->spart : c->spart;
    double* gpart = sb ? sb->gpart : c->gpart;
    const bool want = grad_y != nullptr || grad_T != nullptr;
    if (!want && !sb) {
        // J alone (the autograd function's forward): the plain evaluation with
        // the image-pass kernel of the size rule (the context's scratch holds
        // every variant's partial sums for this grid)
        Level V = P;
        const int v = variant_by_size(V);
        V.variant = variant_ok(V, v) ? v : P.variant;
        const ngf_status e = enqueue_eval(c, V, R, T, y, nullptr);
        if (e != NGF_OK) return e;
        return finish_J(c, J, J_dev);
    }
    if (grad_y) launch_fill(grad_y, 3 * P.Ny(), 0.0f, c->stream);
    if (grad_T) launch_fill(grad_T, P.N(), 0.0f, c->stream);
    ImagePassArgs a = image_args(c, P, R, T, y, want);
    a.gy_atomic = grad_y;
    a.gT_atomic = grad_T;
    a.gscale = gscale;
    a.dpart = dpart;
    a.part = nullptr;
    if (want)
        launch_image_pass_atomic(a, r, P.variant, c->stream);
    else
        launch_image_pass(a, r, P.variant, c->stream);
    HIPCHK(c, hipGetLastError());
    NodePassArgs b{};
    b.y = y;
    b.part = nullptr;
    b.grad = grad_y;
    b.spart = spart;
    b.gpart = gpart;
    b.nx = P.my[0];
    b.ny = P.my[1];
    b.nz = P.my[2];
    int nb[3];
    node_grid(P, nb);
    b.nbx = nb[0];
    b.nby = nb[1];
    b.nbz = nb[2];
    b.cxn = node_chunk(P);
    b.hyx = P.hy[0];
    b.hyy = P.hy[1];
    b.hyz = P.hy[2];
    b.ihy2x = static_cast<float>(1.0 / (P.hy[0] * P.hy[0]));
    b.ihy2y = static_cast<float>(1.0 / (P.hy[1] * P.hy[1]));
    b.ihy2z = static_cast<float>(1.0 / (P.hy[2] * P.hy[2]));
    const double hbary = P.hy[0] * P.hy[1] * P.hy[2];
    b.alpha_hbary = static_cast<float>(c->p.alpha * hbary);
    b.alpha = static_cast<float>(c->p.alpha);
    b.want_grad = grad_y ? 1 : 0;
    b.gather = 0;
    b.gscale = gscale;
    launch_node_pass(b, c->stream);
    HIPCHK(c, hipGetLastError());
    ReduceArgs rd{};
    rd.dpart = dpart;
    rd.nd = static_cast<int>(geometry(P, P.variant).ntiles());
    rd.spart = spart;
    rd.ns = static_cast<int>(node_blocks(P));
    rd.gpart = gpart;
    rd.ng = grad_y ? rd.ns : 0;
    rd.half_hbar = 0.5 * P.h[0] * P.h[1] * P.h[2];
    rd.half_hbary = 0.5 * hbary;
    rd.alpha = c->p.alpha;
    rd.out = c->jds;
    launch_reduce(rd, c->stream);
    HIPCHK(c, hipGetLastError());
    return finish_J(c, J, J_dev);
}

}  // namespace ngf_host

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* ngf_version(void) { return "ngfreg 0.1 gfx950"; }

ngf_status ngf_create(const ngf_params* p, void* stream, ngf_ctx** out) {
    if (!out || !p) return NGF_E_ARG;
    *out = nullptr;
    std::string why;
    if (!params_ok(p, &why)) return NGF_E_ARG;
    ngf_ctx* c = new (std::nothrow) ngf_ctx();
    if (!c) return NGF_E_OOM;
    c->p = *p;
    c->stream = static_cast<hipStream_t>(stream);
    ngf_status s = NGF_OK;
    auto chk = [&](hipError_t e) {
        if (e != hipSuccess && s == NGF_OK) s = NGF_E_HIP;
    };
    chk(hipStreamCreateWithFlags(&c->side[0], hipStreamNonBlocking));
    chk(hipStreamCreateWithFlags(&c->side[1], hipStreamNonBlocking));
    for (int i = 0; i < 3; ++i) chk(hipEventCreateWithFlags(&c->join[i], hipEventDisableTiming));
    chk(hipMalloc(reinterpret_cast<void**>(&c->jds), 8 * sizeof(double)));
    chk(hipHostMalloc(reinterpret_cast<void**>(&c->host_jds),
                      8 * sizeof(double) + sizeof(LbCtl), hipHostMallocDefault));
    chk(hipMalloc(reinterpret_cast<void**>(&c->st), sizeof(LbState)));
    chk(hipMalloc(reinterpret_cast<void**>(&c->dflag), sizeof(int)));
    if (s == NGF_OK) s = static_scratch_setup(c);
    if (s != NGF_OK) {
        ngf_destroy(c);
        return s;
    }
    *out = c;
    return NGF_OK;
}

void ngf_destroy(ngf_ctx* c) {
    if (!c) return;
    if (c->stream || c->side[0]) (void)hipStreamSynchronize(c->stream);
    for (hipStream_t s : c->side)
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
    for (hipEvent_t e : c->join)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev)
        if (e) (void)hipEventDestroy(e);
    free_pyramid(c);
    log_free(c);
    for (void* p : {static_cast<void*>(c->part), static_cast<void*>(c->dpart),
                    static_cast<void*>(c->spart), static_cast<void*>(c->gpart),
                    static_cast<void*>(c->jds), static_cast<void*>(c->dflag),
                    static_cast<void*>(c->ly), static_cast<void*>(c->lg),
                    static_cast<void*>(c->lyt), static_cast<void*>(c->lgt),
                    static_cast<void*>(c->ld), static_cast<void*>(c->ltmp),
                    static_cast<void*>(c->hist), static_cast<void*>(c->st),
                    static_cast<void*>(c->dotpart), static_cast<void*>(c->f64)})
        dfree(p);
    for (void* p : c->pair_owned) dfree(p);
    if (c->host_jds) (void)hipHostFree(c->host_jds);
    delete c;
}

const char* ngf_last_error(const ngf_ctx* c) { return c ? c->err.c_str() : "null context"; }

ngf_status ngf_set_params(ngf_ctx* c, const ngf_params* p) {
    if (!c || !p) return NGF_E_ARG;
    std::string why;
    if (!params_ok(p, &why)) return fail(c, NGF_E_ARG, why);
    if (!c->lv.empty() && (p->levels != c->p.levels || p->ratio != c->p.ratio))
        return fail(c, NGF_E_STATE, "levels and ratio are fixed once a pyramid is built");
    const bool rho_changed = p->rho != c->p.rho;
    c->p = *p;
    if (rho_changed) {
        for (const Level& L : c->lv)
            launch_rn(L.R, L.rn, L.m[0], L.m[1], L.m[2], L.h[0], L.h[1], L.h[2], c->p.rho,
                      c->stream);
        HIPCHK(c, hipGetLastError());
    }
    return NGF_OK;
}

ngf_status ngf_build_pyramid(ngf_ctx* c, const float* R, const float* T, const ngf_grid* g,
                             int32_t host_ptrs) {
    if (!c) return NGF_E_ARG;
    const TraceRange range("ngf_build_pyramid");
    if (!R || !T || !g) return fail(c, NGF_E_ARG, "null R, T or grid");
    const int L = c->p.levels, r = c->p.ratio;
    int64_t N = 1;
    int n0[3];  // level-0 deformation-grid nodes per axis
    for (int d = 0; d < 3; ++d) {
        if (!(std::isfinite(g->h[d]) && g->h[d] > 0.0))
            return fail(c, NGF_E_ARG, "spacing must be positive");
        if (g->m[d] <= 0 || g->m[d] > 32768 || g->m[d] % (1 << (L - 1)) != 0)
            return fail(c, NGF_E_SHAPE,
                        "each m_d must be at most 32768 and divisible by 2^(levels-1)");
        if (c->node_grid[d] == 0 && g->m[d] % (r << (L - 1)) != 0)
            return fail(c, NGF_E_SHAPE, "each m_d must be divisible by ratio * 2^(levels-1)");
        n0[d] = c->node_grid[d] ? c->node_grid[d] : g->m[d] / r + 1;
        if ((n0[d] - 1) % (1 << (L - 1)) != 0)
            return fail(c, NGF_E_SHAPE,
                        "node cells m^y_d - 1 must be divisible by 2^(levels-1)");
        const int mc = g->m[d] >> (L - 1), nc = ((n0[d] - 1) >> (L - 1)) + 1;
        if (mc < 4 || nc < 3)
            return fail(c, NGF_E_SHAPE, "coarsest level needs >= 4 cells and >= 2 node cells");
        if (2 * (n0[d] - 1) > g->m[d])
            return fail(c, NGF_E_SHAPE,
                        "at least 2 image cells per deformation cell: 2 (m^y_d - 1) <= m_d");
        // the image tiles (32 points in y and z) must each meet every index
        // set of Eq. 3 in at most two tiles per axis
        if (g->m[d] > 16 * (n0[d] - 1))
            return fail(c, NGF_E_SHAPE,
                        "at most 16 image cells per deformation cell: m_d <= 16 (m^y_d - 1)");
        N *= g->m[d];
    }
    if (N >= (static_cast<int64_t>(1) << 30))
        return fail(c, NGF_E_SHAPE, "image too large (at most 2^30 - 1 voxels)");
    c->lb_level = -1;
    c->lv.assign(L, Level{});
    for (int l = 0; l < L; ++l) {
        Level& lv = c->lv[l];
        for (int d = 0; d < 3; ++d) {
            lv.m[d] = g->m[d] >> l;
            lv.h[d] = g->h[d] * static_cast<double>(1 << l);
            lv.my[d] = ((n0[d] - 1) >> l) + 1;
            lv.hy[d] = lv.m[d] * lv.h[d] / (lv.my[d] - 1);
        }
        lv.dyadic = 0;
        for (const int q : {2, 4}) {
            bool all = true;
            for (int d = 0; d < 3; ++d) all = all && lv.m[d] % q == 0 && lv.my[d] == lv.m[d] / q + 1;
            if (all) lv.dyadic = q;
        }
        const ngf_status e = bind_level_storage(c, l);
        if (e != NGF_OK) {
            c->lv.clear();
            return e;
        }
    }
    if (const ngf_status st = ensure_scratch(c, c->lv[0]); st != NGF_OK) return st;
    if (ensure_lbfgs(c, static_cast<size_t>(3 * c->lv[0].Ny())) != NGF_OK) return NGF_E_OOM;

    // R on side stream 0, T on side stream 1, each: copy level 0, then the
    // successive 2x2x2 means; both join the context stream.
    const size_t bytes0 = static_cast<size_t>(c->lv[0].N()) * sizeof(float);
    HIPCHK(c, hipEventRecord(c->join[0], c->stream));
    for (int k = 0; k < 2; ++k) {
        hipStream_t s = c->side[k];
        HIPCHK(c, hipStreamWaitEvent(s, c->join[0], 0));
        const float* src = k == 0 ? R : T;
        float* dst0 = k == 0 ? c->lv[0].R : c->lv[0].T;
        HIPCHK(c, hipMemcpyAsync(dst0, src, bytes0,
                                 host_ptrs ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
        for (int l = 1; l < L; ++l) {
            const Level& a = c->lv[l - 1];
            float* out = k == 0 ? c->lv[l].R : c->lv[l].T;
            launch_downsample(k == 0 ? a.R : a.T, out, a.m[0], a.m[1], a.m[2], s);
        }
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipEventRecord(c->join[1 + k], s));
    }
    for (int l = 0; l < L; ++l)
        for (int d = 0; d < 3; ++d)
            launch_index_map(c->lv[l].j0[d], c->lv[l].w0[d], c->lv[l].w1[d], c->lv[l].m[d],
                             c->lv[l].my[d], c->stream);
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->join[1], 0));
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->join[2], 0));
    // reference side of the NGF term, per level (general image pass)
    for (int l = 0; l < L; ++l) {
        const Level& lv = c->lv[l];
        launch_rn(lv.R, lv.rn, lv.m[0], lv.m[1], lv.m[2], lv.h[0], lv.h[1], lv.h[2], c->p.rho,
                  c->stream);
    }
    HIPCHK(c, hipGetLastError());
    // reject non-finite inputs
    int zero = 0;
    HIPCHK(c, hipMemcpyAsync(c->dflag, &zero, sizeof(int), hipMemcpyHostToDevice, c->stream));
    launch_check_finite(c->lv[0].R, c->lv[0].N(), c->dflag, c->stream);
    launch_check_finite(c->lv[0].T, c->lv[0].N(), c->dflag, c->stream);
    int bad = 0;
    HIPCHK(c, hipMemcpyAsync(&bad, c->dflag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (bad) {
        c->lv.clear();
        return fail(c, NGF_E_NONFINITE, "R or T holds NaN or infinity");
    }
    const ngf_status ts = autotune(c);
    if (ts != NGF_OK) return ts;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return NGF_OK;
}

ngf_status ngf_set_kernel(ngf_ctx* c, int32_t variant) {
    if (!c) return NGF_E_ARG;
    if (variant < kVariantBySize || variant >= kNumVariants)
        return fail(c, NGF_E_ARG, "unknown variant");
    c->forced_variant = variant;
    if (!c->lv.empty()) return autotune(c);
    return NGF_OK;
}

ngf_status ngf_set_driver(ngf_ctx* c, int32_t mode) {
    if (!c) return NGF_E_ARG;
    if (mode != 0 && mode != 1) return fail(c, NGF_E_ARG, "mode must be 0 or 1");
    c->host_driven = mode == 1;
    return NGF_OK;
}

ngf_status ngf_set_node_grid(ngf_ctx* c, const int32_t my0[3]) {
    if (!c) return NGF_E_ARG;
    for (int d = 0; d < 3; ++d) {
        const int v = my0 ? my0[d] : 0;
        if (v != 0 && v < 3) return fail(c, NGF_E_ARG, "node counts must be 0 or >= 3");
    }
    for (int d = 0; d < 3; ++d) c->node_grid[d] = my0 ? my0[d] : 0;
    c->lv.clear();  // the next ngf_build_pyramid uses the new grid
    c->lb_level = -1;
    return NGF_OK;
}

ngf_status ngf_set_faults(ngf_ctx* c, int32_t flags) {
    if (!c) return NGF_E_ARG;
    if (flags & ~(NGF_FAULT_REJECT_STEPS | NGF_FAULT_ALLOC))
        return fail(c, NGF_E_ARG, "unknown fault bits");
    c->faults = flags;
    return NGF_OK;
}

ngf_status ngf_get_kernel(const ngf_ctx* c, int32_t level, int32_t* variant) {
    if (!c || !variant) return NGF_E_ARG;
    const ngf_status s = check_level(c, level);
    if (s != NGF_OK) return s;
    *variant = c->lv[level].variant;
    return NGF_OK;
}

ngf_status ngf_level_info(const ngf_ctx* c, int32_t level, ngf_grid* img, ngf_grid* def) {
    if (!c) return NGF_E_ARG;
    const ngf_status s = check_level(c, level);
    if (s != NGF_OK) return s;
    const Level& L = c->lv[level];
    for (int d = 0; d < 3; ++d) {
        if (img) {
            img->m[d] = L.m[d];
            img->h[d] = L.h[d];
        }
        if (def) {
            def->m[d] = L.my[d];
            def->h[d] = L.hy[d];
        }
    }
    return NGF_OK;
}

ngf_status ngf_level_images(ngf_ctx* c, int32_t level, float* R_out, float* T_out) {
    if (!c) return NGF_E_ARG;
    const ngf_status s = check_level(c, level);
    if (s != NGF_OK) return fail(c, s, "no pyramid or bad level");
    const Level& L = c->lv[level];
    const size_t b = static_cast<size_t>(L.N()) * sizeof(float);
    if (R_out) HIPCHK(c, hipMemcpyAsync(R_out, L.R, b, hipMemcpyDeviceToDevice, c->stream));
    if (T_out) HIPCHK(c, hipMemcpyAsync(T_out, L.T, b, hipMemcpyDeviceToDevice, c->stream));
    return NGF_OK;
}

ngf_status ngf_index_map(ngf_ctx* c, int32_t level, int32_t axis, int32_t* j0, float* w0,
                         float* w1) {
    if (!c) return NGF_E_ARG;
    const ngf_status s = check_level(c, level);
    if (s != NGF_OK) return fail(c, s, "no pyramid or bad level");
    if (axis < 0 || axis > 2 || !j0 || !w0 || !w1) return fail(c, NGF_E_ARG, "bad axis or null");
    const Level& L = c->lv[level];
    const size_t m = static_cast<size_t>(L.m[axis]);
    HIPCHK(c, hipMemcpyAsync(j0, L.j0[axis], m * 4, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(w0, L.w0[axis], m * 4, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(w1, L.w1[axis], m * 4, hipMemcpyDeviceToDevice, c->stream));
    return NGF_OK;
}

ngf_status ngf_identity(ngf_ctx* c, int32_t level, float* y) {
    if (!c) return NGF_E_ARG;
    const ngf_status s = check_level(c, level);
    if (s != NGF_OK) return fail(c, s, "no pyramid or bad level");
    if (!y) return fail(c, NGF_E_ARG, "null y");
    const Level& L = c->lv[level];
    launch_identity(y, L.my[0], L.my[1], L.my[2], L.hy[0], L.hy[1], L.hy[2], c->stream);
    HIPCHK(c, hipGetLastError());
    return NGF_OK;
}

ngf_status ngf_eval_J_grad(ngf_ctx* c, int32_t level, const float* y, double* J, float* grad,
                           double* DS) {
    if (!c) return NGF_E_ARG;
    const ngf_status s = check_level(c, level);
    if (s != NGF_OK) return fail(c, s, "no pyramid or bad level");
    if (!y) return fail(c, NGF_E_ARG, "null y");
    const Level& L = c->lv[level];
    ngf_status e = enqueue_eval(c, L, L.R, L.T, y, grad);
    if (e != NGF_OK) return e;
    if (J || DS) {
        if (read_jds(c) != NGF_OK) return NGF_E_HIP;
        if (J) *J = c->host_jds[0];
        if (DS) {
            DS[0] = c->host_jds[1];
            DS[1] = c->host_jds[2];
        }
        if (!std::isfinite(c->host_jds[0])) return fail(c, NGF_E_NONFINITE, "J is not finite");
    }
    return NGF_OK;
}

ngf_status ngf_eval_J_device(ngf_ctx* c, const double** JDS) {
    if (!c || !JDS) return NGF_E_ARG;
    *JDS = c->jds;
    return NGF_OK;
}

ngf_status ngf_lbfgs_reset(ngf_ctx* c, int32_t level, const float* y0) {
    if (!c) return NGF_E_ARG;
    const ngf_status s = check_level(c, level);
    if (s != NGF_OK) return fail(c, s, "no pyramid or bad level");
    if (!y0) return fail(c, NGF_E_ARG, "null y0");
    const Level& L = c->lv[level];
    const size_t n = static_cast<size_t>(3 * L.Ny());
    if (y0 != c->ly)
        HIPCHK(c, hipMemcpyAsync(c->ly, y0, n * sizeof(float), hipMemcpyDeviceToDevice,
                                 c->stream));
    ngf_status e = enqueue_eval(c, L, L.R, L.T, c->ly, c->lg);
    if (e != NGF_OK) return e;
    const double hmin = std::min(L.h[0], std::min(L.h[1], L.h[2]));
    launch_lb_init(c->st, c->p.lbfgs_mem, hmin, c->jds, c->p.max_iter, c->p.early_stop,
                   c->p.tol_J, c->stream);
    HIPCHK(c, hipGetLastError());
    const int reject = (c->faults & NGF_FAULT_REJECT_STEPS) ? 1 : 0;
    HIPCHK(c, hipMemcpyAsync(&c->st->reject_all, &reject, sizeof(int), hipMemcpyHostToDevice,
                             c->stream));
    if (read_jds(c) != NGF_OK) return NGF_E_HIP;
    c->lb_level = level;
    c->lb_J = c->host_jds[0];
    c->lb_gmax = c->host_jds[3];
    c->lb_evals = 1;
    c->lb_iters = 0;
    if (!std::isfinite(c->lb_J)) return fail(c, NGF_E_NONFINITE, "J(y0) is not finite");
    log_start_point(c);
    return NGF_OK;
}

ngf_status ngf_lbfgs_step(ngf_ctx* c, double* J, int32_t* info) {
    if (!c) return NGF_E_ARG;
    const TraceRange range("ngf_lbfgs_step");
    if (c->lb_level < 0 || c->lb_level >= static_cast<int>(c->lv.size()))
        return fail(c, NGF_E_STATE, "ngf_lbfgs_reset first");
    const Level& L = c->lv[c->lb_level];
    const int64_t n = 3 * L.Ny();
    int32_t inf = NGF_INFO_OK;
    if (!std::isfinite(c->lb_gmax)) {
        inf = NGF_INFO_NONFINITE;
    } else if (c->lb_gmax == 0.0) {
        inf = NGF_INFO_CONVERGED;
    } else {
        launch_lb_solve(c->st, c->jds, c->stream);
        launch_lb_combine(c->st, c->hist, static_cast<int64_t>(c->lb_ld), n, c->ly, c->lg, c->ld,
                          c->lyt, c->stream);
        HIPCHK(c, hipGetLastError());
        const double c1 = 1e-4;
        double t = 1.0, gtd = 0.0;
        bool ok = false;
        for (int h = 0; h <= 10; ++h) {
            if (h > 0)
                launch_lb_axpy(c->ly, c->ld, static_cast<float>(t), c->lyt, n, c->stream);
            ngf_status e = enqueue_eval(c, L, L.R, L.T, c->lyt, c->lgt);
            if (e != NGF_OK) return e;
            c->lb_evals++;
            if (read_jds(c) != NGF_OK) return NGF_E_HIP;  // J of the trial and g^T d
            if (h == 0) gtd = c->host_jds[5];
            const double Jt = c->host_jds[0];
            if (armijo_ok(Jt, c->lb_J, c1, t, gtd) && !(c->faults & NGF_FAULT_REJECT_STEPS)) {
                ok = true;
                break;
            }
            t *= 0.5;
        }
        if (!ok) {
            inf = NGF_INFO_LINESEARCH_FAIL;
        } else {
            const int nb = lb_dot_blocks(n);
            launch_lb_update_dots(c->st, c->hist, static_cast<int64_t>(c->lb_ld), n, c->ly, c->lyt,
                                  c->lg, c->lgt, c->dotpart, nb, c->p.lbfgs_mem, c->stream);
            launch_lb_gram_update(c->st, c->dotpart, nb, c->jds, c->stream);
            HIPCHK(c, hipGetLastError());
            std::swap(c->ly, c->lyt);
            std::swap(c->lg, c->lgt);
            c->lb_J = c->host_jds[0];
            c->lb_gmax = c->host_jds[3];
            c->lb_iters++;
            log_host_step(c, t);
        }
    }
    if (J) *J = c->lb_J;
    if (info) *info = inf;
    return NGF_OK;
}

ngf_status ngf_lbfgs_get(ngf_ctx* c, float* y, float* grad, double* J) {
    if (!c) return NGF_E_ARG;
    if (c->lb_level < 0) return fail(c, NGF_E_STATE, "ngf_lbfgs_reset first");
    const size_t n = static_cast<size_t>(3 * c->lv[c->lb_level].Ny());
    if (y) HIPCHK(c, hipMemcpyAsync(y, c->ly, n * 4, hipMemcpyDeviceToDevice, c->stream));
    if (grad) HIPCHK(c, hipMemcpyAsync(grad, c->lg, n * 4, hipMemcpyDeviceToDevice, c->stream));
    if (J) *J = c->lb_J;
    return NGF_OK;
}

ngf_status ngf_prolongate(ngf_ctx* c, int32_t coarse_level, const float* y_c, float* y_f) {
    if (!c) return NGF_E_ARG;
    const ngf_status s = check_level(c, coarse_level);
    if (s != NGF_OK) return fail(c, s, "no pyramid or bad level");
    if (coarse_level == 0) return fail(c, NGF_E_LEVEL, "level 0 has no finer level");
    if (!y_c || !y_f) return fail(c, NGF_E_ARG, "null pointer");
    const Level& C = c->lv[coarse_level];
    const Level& F = c->lv[coarse_level - 1];
    for (int d = 0; d < 3; ++d)
        if (F.my[d] - 1 != 2 * (C.my[d] - 1))
            return fail(c, NGF_E_SHAPE, "grids are not 2:1 aligned");
    launch_prolongate(y_c, y_f, C.my[0], C.my[1], C.my[2], c->stream);
    HIPCHK(c, hipGetLastError());
    return NGF_OK;
}

ngf_status ngf_register_levels(ngf_ctx* c, float* y_out, ngf_report* rep) {
    if (!c) return NGF_E_ARG;
    if (c->lv.empty()) return fail(c, NGF_E_STATE, "no pyramid");
    if (rep) {
        std::memset(rep, 0, sizeof(*rep));
        rep->levels = static_cast<int32_t>(c->lv.size());
    }
    c->log.clear();
    const int L = static_cast<int>(c->lv.size());
    for (int lev = L - 1; lev >= 0; --lev) {
        char rname[64];
        std::snprintf(rname, sizeof(rname), "ngf level %d (%dx%dx%d)", lev, c->lv[lev].m[0],
                      c->lv[lev].m[1], c->lv[lev].m[2]);
        const TraceRange range(rname);
        const auto t_level = std::chrono::steady_clock::now();
        const Level& lv = c->lv[lev];
        if (lev == L - 1) {
            launch_identity(c->ltmp, lv.my[0], lv.my[1], lv.my[2], lv.hy[0], lv.hy[1], lv.hy[2],
                            c->stream);
        } else {
            const Level& C = c->lv[lev + 1];
            launch_prolongate(c->ly, c->ltmp, C.my[0], C.my[1], C.my[2], c->stream);
        }
        HIPCHK(c, hipGetLastError());
        ngf_status e = ngf_lbfgs_reset(c, lev, c->ltmp);
        if (e != NGF_OK) return e;
        int it = 0;
        int32_t info = NGF_INFO_MAX_ITER;
        if (c->host_driven) {
            while (it < c->p.max_iter) {
                const double J_old = c->lb_J;
                int32_t inf = 0;
                double Jn = 0.0;
                e = ngf_lbfgs_step(c, &Jn, &inf);
                if (e != NGF_OK) return e;
                if (inf != NGF_INFO_OK) {
                    info = inf;
                    break;
                }
                ++it;
                if (c->p.early_stop && early_stop_met(J_old, Jn, c->p.tol_J)) {
                    info = NGF_INFO_CONVERGED;
                    break;
                }
            }
        } else {
            LbCtl ctl{};
            e = run_level_on_device(c, &ctl);
            if (e != NGF_OK) return e;
            it = ctl.iters;
            info = ctl.info;
        }
        if (rep) {
            HIPCHK(c, hipStreamSynchronize(c->stream));
            rep->ms[lev] = std::chrono::duration<double, std::milli>(
                               std::chrono::steady_clock::now() - t_level)
                               .count();
            rep->iters[lev] = it;
            rep->evals[lev] = c->lb_evals;
            rep->J[lev] = c->lb_J;
            rep->info[lev] = info;
        }
    }
    if (y_out) {
        const size_t n = static_cast<size_t>(3 * c->lv[0].Ny());
        HIPCHK(c, hipMemcpyAsync(y_out, c->ly, n * 4, hipMemcpyDeviceToDevice, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return NGF_OK;
}

ngf_status ngf_register(ngf_ctx* c, const float* R, const float* T, const ngf_grid* g,
                        float* y_out, int32_t host_ptrs, ngf_report* rep) {
    if (!c) return NGF_E_ARG;
    const TraceRange range("ngf_register");
    ngf_status e = ngf_build_pyramid(c, R, T, g, host_ptrs);
    if (e != NGF_OK) return e;
    if (!host_ptrs) return ngf_register_levels(c, y_out, rep);
    e = ngf_register_levels(c, nullptr, rep);
    if (e != NGF_OK) return e;
    if (y_out) {
        const size_t n = static_cast<size_t>(3 * c->lv[0].Ny());
        HIPCHK(c, hipMemcpyAsync(y_out, c->ly, n * 4, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return NGF_OK;
}

ngf_status ngf_apply_P(ngf_ctx* c, int32_t level, const float* y, float* yhat) {
    if (!c) return NGF_E_ARG;
    const ngf_status s = check_level(c, level);
    if (s != NGF_OK) return fail(c, s, "no pyramid or bad level");
    if (!y || !yhat) return fail(c, NGF_E_ARG, "null pointer");
    const Level& L = c->lv[level];
    launch_apply_P(L.j0, L.w0, L.w1, L.m, L.my, y, yhat, c->stream);
    HIPCHK(c, hipGetLastError());
    return NGF_OK;
}

ngf_status ngf_apply_PT(ngf_ctx* c, int32_t level, const float* z, float* out, int32_t scheme) {
    if (!c) return NGF_E_ARG;
    const ngf_status s = check_level(c, level);
    if (s != NGF_OK) return fail(c, s, "no pyramid or bad level");
    if (!z || !out) return fail(c, NGF_E_ARG, "null pointer");
    if (scheme < 0 || scheme > 2) return fail(c, NGF_E_ARG, "scheme must be 0, 1 or 2");
    const Level& L = c->lv[level];
    if (scheme != 0) launch_fill(out, 3 * L.Ny(), 0.0f, c->stream);
    launch_apply_PT(L.j0, L.w0, L.w1, L.m, L.my, z, out, scheme, c->stream);
    HIPCHK(c, hipGetLastError());
    return NGF_OK;
}

ngf_status ngf_set_profiling(ngf_ctx* c, int32_t enable, int32_t level) {
    if (!c) return NGF_E_ARG;
    c->prof_only = level < 0 ? -1 : level;
    if (enable && c->ev.empty()) {
        c->ev.resize(2 * kProfMax, nullptr);
        for (auto& e : c->ev) HIPCHK(c, hipEventCreate(&e));
        c->prof_level.assign(kProfMax, -1);
    }
    c->prof = enable != 0;
    c->nprof = 0;
    return NGF_OK;
}

ngf_status ngf_kernel_time(ngf_ctx* c, int32_t level, int32_t* launches, double* total_ms,
                           int64_t* voxels, int64_t* nodes) {
    if (!c) return NGF_E_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double tot = 0.0;
    int n = 0;
    int64_t vox = 0, nod = 0;
    for (int i = 0; i < c->nprof; ++i) {
        const int l = c->prof_level[i];
        if (level >= 0 && l != level) continue;
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]));
        tot += ms;
        ++n;
        if (l >= 0 && l < static_cast<int>(c->lv.size())) {
            vox += c->lv[l].N();
            nod += c->lv[l].Ny();
        } else {
            vox += c->pair.N();
            nod += c->pair.Ny();
        }
    }
    if (launches) *launches = n;
    if (total_ms) *total_ms = tot;
    if (voxels) *voxels = vox;
    if (nodes) *nodes = nod;
    c->nprof = 0;
    return NGF_OK;
}

ngf_status ngf_eval_pair(ngf_ctx* c, const ngf_grid* g, const int32_t my[3], const float* R,
                         const float* T, const float* y, const double* gscale, double* J,
                         double* J_dev, float* grad_y, float* grad_T) {
    if (!c) return NGF_E_ARG;
    if (!g || !my || !R || !T || !y) return fail(c, NGF_E_ARG, "null argument");
    const int r = c->p.ratio;
    int64_t N = 1;
    for (int d = 0; d < 3; ++d) {
        if (!(std::isfinite(g->h[d]) && g->h[d] > 0.0)) return fail(c, NGF_E_ARG, "bad spacing");
        if (g->m[d] < 4 || g->m[d] % r != 0 || my[d] != g->m[d] / r + 1)
            return fail(c, NGF_E_SHAPE, "need m_d >= 4, divisible by ratio, my_d = m_d/ratio + 1");
        N *= g->m[d];
    }
    if (N >= (static_cast<int64_t>(1) << 31)) return fail(c, NGF_E_SHAPE, "image too large");
    Level& P = c->pair;
    bool same = true;
    for (int d = 0; d < 3; ++d) same = same && P.m[d] == g->m[d] && P.h[d] == g->h[d];
    if (!same || P.j0[0] == nullptr) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (void* p : c->pair_owned) dfree(p);
        c->pair_owned.clear();
        for (int d = 0; d < 3; ++d) {
            P.m[d] = g->m[d];
            P.h[d] = g->h[d];
            P.my[d] = my[d];
            P.hy[d] = P.m[d] * P.h[d] / (P.my[d] - 1);
            if (dalloc(c, &P.j0[d], P.m[d]) != NGF_OK || dalloc(c, &P.w0[d], P.m[d]) != NGF_OK ||
                dalloc(c, &P.w1[d], P.m[d]) != NGF_OK)
                return NGF_E_OOM;
            c->pair_owned.push_back(P.j0[d]);
            c->pair_owned.push_back(P.w0[d]);
            c->pair_owned.push_back(P.w1[d]);
            launch_index_map(P.j0[d], P.w0[d], P.w1[d], P.m[d], P.my[d], c->stream);
        }
        HIPCHK(c, hipGetLastError());
    }
    P.variant = kScatterVariant;  // the scatter form lives in a 3D-tile kernel
    P.dyadic = r;
    if (const ngf_status st = ensure_scratch(c, P); st != NGF_OK) return st;
    return eval_scatter(c, P, R, T, y, gscale, J, J_dev, grad_y, grad_T, nullptr);
}

ngf_status ngf_eval_J_grad_T(ngf_ctx* c, int32_t level, const float* y, const double* gscale,
                             double* J, double* J_dev, float* grad_y, float* grad_T) {
    if (!c) return NGF_E_ARG;
    const ngf_status s = check_level(c, level);
    if (s != NGF_OK) return fail(c, s, "no pyramid or bad level");
    if (!y) return fail(c, NGF_E_ARG, "null y");
    const Level& L = c->lv[level];
    if (!L.dyadic)
        return fail(c, NGF_E_SHAPE,
                    "the scatter form needs a deformation grid of m/2 + 1 or m/4 + 1 nodes");
    Level P = L;  // same grids and buffers; the scatter lives in a 3D-tile kernel
    P.variant = kScatterVariant;
    return eval_scatter(c, P, L.R, L.T, y, gscale, J, J_dev, grad_y, grad_T, nullptr);
}

}  // extern "C"
