// Internal declarations shared by the HIP kernels and the host side of the
// library.  Not part of the public ABI (include/ngfreg.h is).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/ngfreg.h"
#include <stdint.h>

namespace ngf {

constexpr int kThreads = 256;      // threads per workgroup (four wave64s)
constexpr int kMaxMem = 8;         // largest L-BFGS memory
constexpr int kSlots = kMaxMem + 1;             // ring slots (one spare)
constexpr int kBasis = 2 * kSlots + 1;          // s slots, t slots, gradient
constexpr int kBasisG = 2 * kSlots;             // basis index of the gradient

// Image-pass tile (voxels per axis).  Tiles are aligned to the deformation
// grid: each extent is a multiple of the grid ratio.
constexpr int kTX = 8, kTY = 8, kTZ = 32;
// Marching image pass: (y, z) tile of kMY x (32 or 64); the x chunk is a
// run-time choice.
constexpr int kMY = 16;
// Node pass: (y, z) tile of kNMY x kNMZ nodes, marching along x in a chunk
// fitted to the grid and the device.
constexpr int kNMY = 8, kNMZ = 32;
constexpr int kNodeChunkMax = 256;  // node planes per node-pass workgroup, at most

// Image-pass variants the autotuner chooses from: the 3D-tile kernel at three
// tile sizes, and the marching kernel with in-plane tile 16 x 64 or 16 x 32
// and x chunks of 8, 16, 20 or 32 planes, or of a length fitted to the level
// and the device (the "fit" variants: see fit_chunk).
enum Variant {
    kTile3D = 0,
    kMarch64x8 = 1, kMarch64x20 = 2, kMarch64x32 = 3,
    kMarch32x8 = 4, kMarch32x20 = 5, kMarch32x32 = 6,
    kTile3DSmall = 7,  // 3D tile of 4 x 8 x 32 voxels (coarse levels)
    kTile3DTiny = 8,   // 3D tile of 4 x 4 x 16 voxels (many workgroups for small levels)
    kMarch64x16 = 9, kMarch32x16 = 10,
    kMarch32Fit = 11, kMarch64Fit = 12,
    kMarchSqFit = 13,  // 32 x 32 (y, z) tile, 512-thread workgroups, fitted x chunk
    kMarchGen = 14,    // general index maps, 32 x 32 tile, one barrier per plane
    kNumVariants = 15
};
constexpr int kVariantBySize = -2;  // selection rule instead of timed selection
inline bool is_march(int v) {
    return (v >= kMarch64x8 && v <= kMarch32x32) || (v >= kMarch64x16 && v <= kMarchSqFit);
}
inline bool is_gen(int v) { return v == kMarchGen; }
// 3D-tile extents (x, y, z) of the 3D-tile variants
inline int tile3d_x(int v) { return v == kTile3D ? 8 : 4; }
inline int tile3d_y(int v) { return v == kTile3DTiny ? 4 : 8; }
inline int tile3d_z(int v) { return v == kTile3DTiny ? 16 : 32; }
inline bool is_tile3d(int v) { return v == kTile3D || v == kTile3DSmall || v == kTile3DTiny; }
// 3D tile of the differentiation form (float atomics into grad_y and grad_T):
// four voxels per thread keep the warp cells they scatter from in fewer
// registers than the 8 x 8 x 32 tile's eight
constexpr int kScatterVariant = kTile3DSmall;
// fixed x chunk of a marching variant; 0 for the fit variants
inline int march_cx(int v) {
    if (v >= kMarch32Fit) return 0;
    if (v >= kMarch64x16) return 16;
    return (v - 1) % 3 == 0 ? 8 : ((v - 1) % 3 == 1 ? 20 : 32);
}
inline int march_tz(int v) {
    return (v <= kMarch64x32 || v == kMarch64x16 || v == kMarch64Fit) ? 64 : 32;
}
inline int march_ty(int v) { return (v == kMarchSqFit || v == kMarchGen) ? 32 : kMY; }
// variants whose kernels hold a grid ratio of 2 or 4 in their code (the
// general pass reads the index maps and takes any ratio >= 2)
inline bool needs_dyadic(int v) { return v != kMarchGen; }
// Workgroups of the marching kernel with (y, z) tile ty x tz that the
// current device holds at once (occupancy per CU times the CU count).
int image_march_slots(int ty, int tz);
// Chunk length along x for a launch of `across` x-columns of workgroups over
// an axis of `len` planes: the multiple of `step` (at least `lo`) that
// minimises the launch's predicted duration, taken as the number of full
// rounds of workgroups over the `slots` the device holds at once times the
// planes a workgroup walks (its chunk plus four lead-in and lead-out steps).
// A chunk that fills the slots once beats a shorter one that needs a partly
// empty last round.
inline int fit_chunk(int len, int64_t across, int step, int lo, int slots, int hi = 1 << 30) {
    int top = ((len + step - 1) / step) * step;
    if (top > hi) top = hi;
    int best = lo;
    int64_t best_cost = -1;
    for (int cx = lo; cx <= (top > lo ? top : lo); cx += step) {
        const int64_t n = across * ((len + cx - 1) / cx);
        const int64_t cost = ((n + slots - 1) / slots) * (cx + 4);
        if (best_cost < 0 || cost < best_cost) best = cx, best_cost = cost;
    }
    return best;
}
// Workgroups of the marching node pass the current device holds at once.
int node_march_slots();
// Workgroups of the general marching image pass the device holds at once.
int image_gen_slots();

// Index maps of the grid conversion along one axis of m image cells and n
// nodes (Sec. 2.2, "Grid conversion"): image point i lies at node coordinate
// (2i+1)(n-1)/(2m), so its lower node is j0(i) = (2i+1)(n-1) div 2m.
// first_at_least(k) is the smallest i with j0(i) >= k (m when there is none).
// Exact in 32-bit integers for m <= 32768 (checked by the host).
__host__ __device__ inline int map_lower(int i, int m, int n) {
    return ((2 * i + 1) * (n - 1)) / (2 * m);
}
__host__ __device__ inline int first_at_least(int k, int m, int n) {
    if (k <= 0) return 0;
    const int c = (2 * m * k + (n - 2)) / (n - 1);  // ceil(2 m k / (n - 1))
    const int i = c / 2;                            // ceil((c - 1) / 2)
    return i < m ? i : m;
}
// Image tiles of extent te along an axis that hold node j in their blocks of
// P^T partial sums: the tiles of the first and the last image point of the
// node's index set (Eq. 3), and the node's place in each block (a tile's
// block starts at the lower node of the tile's first point).  tb < 0: one
// tile.
struct NodeTiles {
    int ta, la, tb, lb;
};
__host__ __device__ inline NodeTiles node_tiles(int j, int m, int n, int te) {
    const int ilo = first_at_least(j - 1, m, n);
    const int ihi = first_at_least(j + 1, m, n) - 1;
    NodeTiles r;
    r.ta = ilo / te;
    r.la = j - map_lower(r.ta * te, m, n);
    const int tb = ihi / te;
    r.tb = tb != r.ta ? tb : -1;
    r.lb = tb != r.ta ? j - map_lower(tb * te, m, n) : 0;
    return r;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Renumbering gives each XCD a contiguous range of tiles, so that
// neighbouring tiles (which share halo data) meet in the same L2: XCD x
// (= b mod 8) receives blocks x, x + 8, ..., i.e. q + (x < r) of them for
// n = 8 q + r, and they take the tiles from x q + min(x, r) on.  A bijection
// of [0, n) for every n.
__host__ __device__ inline int xcd_tile(int b, int n) {
    const int x = b & 7, q = n >> 3, r = n & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// One pyramid level as the kernels see it.
struct LevelView {
    int m[3];          // image cells
    int my[3];         // deformation nodes
    double h[3];       // image spacing
    double hy[3];      // node spacing
    const float* R;
    const float* T;
    const int32_t* j0[3];  // index maps (per axis, m entries)
    const float* w0[3];
    const float* w1[3];
};

struct ImagePassArgs {
    const float* R;
    const float* T;
    const float* y;        // [3][my]
    const int32_t* j0x; const int32_t* j0y; const int32_t* j0z;
    const float* w0x; const float* w0y; const float* w0z;
    const float* w1x; const float* w1y; const float* w1z;
    const float4* rn;      // reference side of the NGF term per voxel (general pass)
    float* part;           // P^T partial sums per tile, [tile][3][px][py][pz]
    double* dpart;         // sum over the tile of (1 - r^2), one per tile
    int mx, my, mz;        // image cells
    int nx, ny, nz;        // deformation nodes
    int ntx, nty, ntz;     // tiles per axis
    int cx;                // x chunk of the marching form (image planes)
    int px, py, pz;        // nodes per tile block of the P^T partial sums, per axis
    double hx, hy, hz;     // spacing (float64: continuous index of the warp)
    double ihx, ihy, ihz;  // 1 / h, used only when every h is a power of two
    int pow2h;             // 1: every spacing is a power of two (exact reciprocal)
    float fihx, fihy, fihz;        // 1 / h in float32
    float i2hx, i2hy, i2hz;        // 1 / (2 h)
    float tau, rho;
    float hbar;            // h_x h_y h_z
    int want_grad;         // 0: value only
    // differentiation form: P^T and dJ/dT by atomic scatter (null: not wanted)
    float* gy_atomic;      // [3][my], accumulated in place (zeroed beforehand)
    float* gT_atomic;      // [mx][my][mz], accumulated in place (zeroed beforehand)
    const double* gscale;  // device scalar multiplying both (null: 1)
    const int* gate;       // device flag: the pass does nothing when *gate == kOpNone (null: always run)
};

struct NodePassArgs {
    const float* y;        // [3][my]
    const float* part;     // image-pass partial sums
    float* grad;           // [3][my] output (may be null when want_grad == 0)
    double* spart;         // per block: sum of (A u)^2
    double* gpart;         // per block: [0] max |grad|, [1] sum grad^2
    int nx, ny, nz;
    int ntx, nty, ntz;     // image-pass tiles per axis
    int tex, tey, tez;     // image-pass tile extent per axis (voxels)
    int mx, my, mz;        // image cells per axis (for the index maps)
    int px, py, pz;        // nodes per tile block of the image-pass partial sums
    int nbx, nby, nbz;     // node-pass blocks per axis
    int cxn;               // x chunk of the marching form (node planes)
    double hyx, hyy, hyz;  // node spacing (float64, for X = j h^y)
    float ihy2x, ihy2y, ihy2z;  // 1 / (h^y)^2
    float alpha_hbary;     // alpha * hbar^y
    float alpha;
    int want_grad;
    int gather;            // 1: sum the image-tile partials; 0: grad already holds grad D
    const double* gscale;  // device scalar multiplying alpha grad S when gather == 0
    const int* gate;       // as in ImagePassArgs
};

struct LbState;

struct ReduceArgs {
    const double* dpart; int nd;
    const double* spart; int ns;
    const double* gpart; int ng;   // pairs (max, sumsq); ng == 0: skip
    double half_hbar, half_hbary, alpha;
    double* out;                    // {J, D, S, max|g|, |g|^2}
    const int* gate;                // as in ImagePassArgs
    LbState* lb;                    // device-driven level: Armijo test of J (null: none)
};

// L-BFGS device state; lives in device memory, read and written by the
// vector kernels and the single-thread solver.
// Device-driven L-BFGS level: the line search as a state machine that the
// kernels of one round (plan, vector update, evaluation, decision, history
// update) advance, so that the host can enqueue rounds without reading
// anything back in between.
enum LbPhase : int { kPhNeedDir = 0, kPhTrial = 1, kPhAccepted = 2, kPhDone = 3 };
enum LbOp : int { kOpNone = 0, kOpCombine = 1, kOpAxpy = 2 };
constexpr int kRoundBatch = 16;  // rounds enqueued between reads of the control block
struct LbCtl {
    int op;          // what the current round's vector kernel does (first: the gate)
    int phase;
    int halvings;    // rejected trials along the current direction
    int iters;       // accepted steps on this level
    int evals;       // evaluations on this level (the start point's included)
    int info;        // NGF_INFO_* once phase == kPhDone
    int max_iter;
    int early_stop;
    double t;        // trial step length
    double tol;      // early-stop tolerance
    double J;        // objective at the current point
    double gmax;     // max |grad J| at the current point
};

struct LbState {
    LbCtl ctl;                      // read back by the host between batches of rounds
    double J, D, S, gmax, gnorm2;   // copy of the last evaluation
    double gtd;                     // g^T d of the current direction
    double flags;                   // bit 0: memory reset, bit 1: zero gradient
    double count_d;                 // stored pairs (as double, for the host)
    // device-only:
    int count;
    int order[kSlots];              // slots of stored pairs, oldest first
    int free_slot;
    int mem;
    double hmin;
    double G[kBasis * kBasis];      // inner products of the basis vectors
    double coef[kBasis];            // direction coefficients over the basis
    int reject_all;                 // failure injection: every trial fails the Armijo test
};

__device__ inline void lb_finish(LbCtl& c, int info) {
    c.phase = kPhDone;
    c.info = info;
    c.op = kOpNone;
}

// Armijo test of the trial just evaluated, objective Jt (c1 = 1e-4, at most
// 10 halvings).  Contraction is off so that the test rounds exactly as the
// host's.  One lane; no-op when the round had no trial.
__device__ inline void lb_decide_one(LbState* st, double Jt) {
#pragma clang fp contract(off)
    LbCtl& c = st->ctl;
    if (c.op == kOpNone) return;
    c.evals += 1;
    const double c1 = 1e-4;
    if (isfinite(Jt) && Jt <= c.J + c1 * c.t * st->gtd && !st->reject_all) {
        c.phase = kPhAccepted;
    } else {
        c.t *= 0.5;
        c.halvings += 1;
        if (c.halvings > 10) lb_finish(c, NGF_INFO_LINESEARCH_FAIL);
    }
}

// ---------------------------------------------------------------------------
// Batched launches: one launch covers the same stage of many independent
// pairs.  A block table maps each workgroup to (pair, block index within the
// pair's own launch); pair < 0 marks padding.  Each pair's range of the table
// starts at a multiple of 8, so every block lands on the XCD it would have in
// the pair's own launch.  The bodies are those of the single-pair kernels,
// so every pair computes exactly what its own launch computes.
// ---------------------------------------------------------------------------
struct BlockRef {
    int pair;
    int block;
};

// one pair's L-BFGS buffers for the batched round kernels
struct LbVecArgs {
    LbState* st;
    float* hist;
    int64_t ld;
    int64_t n;
    float* y;
    float* g;
    float* d;
    float* yt;
    float* gt;
    double* dotpart;
    int nblocks;      // blocks of the pair's vector launches (lb_dot_blocks(n))
    double* jds;
    // level start
    int mem, max_iter, early_stop;
    double hmin, tol;
};

void launch_image_pass_batch(const ImagePassArgs* args, const BlockRef* blk, int nblk, int ratio,
                             int variant, bool pow2, hipStream_t s);
void launch_image_march_batch(const ImagePassArgs* args, const BlockRef* blk, int nblk,
                              int ratio, int variant, bool pow2, hipStream_t s);
void launch_node_pass_batch(const NodePassArgs* args, const BlockRef* blk, int nblk,
                            hipStream_t s);
void launch_reduce_batch(const ReduceArgs* args, int npairs, hipStream_t s);
void launch_lb_init_batch(const LbVecArgs* args, int npairs, hipStream_t s);
void launch_lb_plan_batch(const LbVecArgs* args, int npairs, hipStream_t s);
void launch_lb_vec_batch(const LbVecArgs* args, const BlockRef* blk, int nblk, hipStream_t s);
void launch_lb_accept_batch(const LbVecArgs* args, const BlockRef* blk, int nblk, int npairs,
                            int mem, hipStream_t s);
void launch_ctl_gather(const LbVecArgs* args, LbCtl* out, int npairs, hipStream_t s);

// kernels (definitions in the .hip files), launched from the host code
void launch_downsample(const float* src, float* dst, int mx, int my, int mz, hipStream_t s);
void launch_index_map(int32_t* j0, float* w0, float* w1, int m, int my, hipStream_t s);
void launch_identity(float* y, int nx, int ny, int nz, double hx, double hy, double hz,
                     hipStream_t s);
void launch_prolongate(const float* yc, float* yf, int cx, int cy, int cz, hipStream_t s);
void launch_image_pass(const ImagePassArgs& a, int ratio, int variant, hipStream_t s);
void launch_image_march(const ImagePassArgs& a, int ratio, int ty, int tz, int cx,
                        hipStream_t s);
void launch_image_gen(const ImagePassArgs& a, int cx, hipStream_t s);
void launch_image_gen_batch(const ImagePassArgs* args, const BlockRef* blk, int nblk, bool pow2,
                            hipStream_t s);
void launch_rn(const float* R, float4* rn, int mx, int my, int mz, double hx, double hy,
               double hz, double rho, hipStream_t s);
void launch_node_pass(const NodePassArgs& a, hipStream_t s);
void launch_reduce(const ReduceArgs& a, hipStream_t s);
void launch_check_finite(const float* v, int64_t n, int* flag, hipStream_t s);
void launch_fill(float* p, int64_t n, float v, hipStream_t s);
void launch_image_pass_atomic(const ImagePassArgs& a, int ratio, int variant, hipStream_t s);

// standalone grid conversion (P, and P^T by gather / atomic scatter / red-black)
void launch_apply_P(const int32_t* const j0[3], const float* const w0[3],
                    const float* const w1[3], const int m[3], const int n[3], const float* y,
                    float* yh, hipStream_t s);
void launch_apply_PT(const int32_t* const j0[3], const float* const w0[3],
                     const float* const w1[3], const int m[3], const int n[3], const float* z,
                     float* out, int scheme, hipStream_t s);

// L-BFGS vector kernels
void launch_lb_solve(LbState* st, double* jds, hipStream_t s);
// one round of the device-driven level (see LbCtl): the plan of the first
// round, then per round vec, evaluation, accept; accept ends with the plan of
// the next round
void launch_lb_plan(LbState* st, double* jds, hipStream_t s);
void launch_lb_vec(LbState* st, const float* hist, int64_t ld, int64_t n, const float* y,
                   const float* g, float* d, float* yt, hipStream_t s);
void launch_lb_accept(LbState* st, float* hist, int64_t ld, int64_t n, float* y,
                      const float* yt, float* g, const float* gt, double* dotpart,
                      int nblocks, double* jds, int mem, hipStream_t s);
void launch_lb_combine(LbState* st, const float* hist, int64_t ld, int64_t n, const float* y,
                       const float* g, float* d, float* yt, hipStream_t s);
void launch_lb_axpy(const float* y, const float* d, float t, float* yt, int64_t n,
                    hipStream_t s);
void launch_lb_update_dots(LbState* st, float* hist, int64_t ld, int64_t n, const float* y,
                           const float* yt, const float* g, const float* gt,
                           double* dotpart, int nblocks, int mem, hipStream_t s);
void launch_lb_gram_update(LbState* st, const double* dotpart, int nblocks,
                           const double* jds, hipStream_t s);
void launch_lb_init(LbState* st, int mem, double hmin, const double* jds, int max_iter,
                    int early_stop, double tol, hipStream_t s);
int lb_dot_blocks(int64_t n);


}  // namespace ngf
