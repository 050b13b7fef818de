// The no-allocation variant of the differentiation form (ngf_eval_pair): its
// scratch -- the pair's index maps and the partial sums of D, S and the
// gradient norms -- lives in one static device array instead of buffers the
// context allocates, for callers that cannot allocate (graph capture, tight
// serving loops).  The kernels are those of ngf_eval_pair.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "../../include/ngfreg.h"
#include "ngf_ctx.h"
#include "ngf_internal.h"

using namespace ngf;
using namespace ngf_host;

namespace {

constexpr size_t kScratchBytes = size_t{2} << 20;  // 2 MiB per device
constexpr int kMaxDevices = 64;

// Each device holds its own copy until the process ends.  Host code never
// passes this name to a kernel: it uses the address taken per device below.
__device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

namespace ngf_host {

ngf_status static_scratch_setup(ngf_ctx* c) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(c, NGF_E_HIP, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices) return fail(c, NGF_E_HIP, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[dev]) return NGF_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
        (void)hipGetLastError();
        return fail(c, NGF_E_HIP,
                    std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    }
    g_ptr[dev] = p;
    return NGF_OK;
}

}  // namespace ngf_host

extern "C" ngf_status ngf_eval_pair_static(ngf_ctx* c, const ngf_grid* g, const int32_t my[3],
                                           const float* R, const float* T, const float* y,
                                           const double* gscale, double* J, double* J_dev,
                                           float* grad_y, float* grad_T) {
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
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(c, NGF_E_HIP, "hipGetDevice failed");
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        base = g_ptr[dev];
    }
    if (!base) return fail(c, NGF_E_STATE, "static scratch not set up on this device");

    Level P;
    for (int d = 0; d < 3; ++d) {
        P.m[d] = g->m[d];
        P.h[d] = g->h[d];
        P.my[d] = my[d];
        P.hy[d] = P.m[d] * P.h[d] / (P.my[d] - 1);
    }
    P.variant = kScatterVariant;  // the scatter form lives in a 3D-tile kernel
    P.dyadic = r;
    // layout of the scratch: D partials per image tile, S partials and
    // (max, sum of squares) of the gradient per node block, then the index
    // maps (j0, w0, w1 per axis)
    const size_t nt = static_cast<size_t>(geometry(P, kScatterVariant).ntiles());
    const size_t nb = static_cast<size_t>(node_blocks(P));
    size_t off = 0;
    const size_t o_d = off;
    off = align256(off + nt * sizeof(double));
    const size_t o_s = off;
    off = align256(off + nb * sizeof(double));
    const size_t o_g = off;
    off = align256(off + 2 * nb * sizeof(double));
    size_t o_map[3][3];
    for (int d = 0; d < 3; ++d)
        for (int k = 0; k < 3; ++k) {
            o_map[d][k] = off;
            off = align256(off + static_cast<size_t>(P.m[d]) * 4);
        }
    if (off > kScratchBytes)
        return fail(c, NGF_E_SHAPE,
                    "grid too large for the static scratch of the no-allocation form (" +
                        std::to_string(off) + " bytes needed, 2 MiB available)");
    char* s = static_cast<char*>(base);
    for (int d = 0; d < 3; ++d) {
        P.j0[d] = reinterpret_cast<int32_t*>(s + o_map[d][0]);
        P.w0[d] = reinterpret_cast<float*>(s + o_map[d][1]);
        P.w1[d] = reinterpret_cast<float*>(s + o_map[d][2]);
        launch_index_map(P.j0[d], P.w0[d], P.w1[d], P.m[d], P.my[d], c->stream);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, NGF_E_HIP, hipGetErrorString(e));
    const ScatterBufs sb{reinterpret_cast<double*>(s + o_d), reinterpret_cast<double*>(s + o_s),
                         reinterpret_cast<double*>(s + o_g)};
    return eval_scatter(c, P, R, T, y, gscale, J, J_dev, grad_y, grad_T, &sb);
}
