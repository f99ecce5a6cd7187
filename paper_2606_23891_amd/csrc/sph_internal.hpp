// Shared internals of libsph: plan tables, launch-argument structs, error
// reporting and wave-level helpers for gfx950 (wave64).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sph.h"
#include "sph_layouts.hpp"

namespace sph {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
sph_status fail(sph_status s, const std::string &msg);
sph_status hip_fail(hipError_t e, const char *what);

#define SPH_HIP(call)                                        \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return ::sph::hip_fail(e_, #call); \
    } while (0)

#define SPH_CHECK_LAUNCH(what)                               \
    do {                                                     \
        hipError_t e_ = hipGetLastError();                   \
        if (e_ != hipSuccess) return ::sph::hip_fail(e_, what); \
    } while (0)

// ---------------------------------------------------------------------------
// plan tables (device copies are plain arrays of these)
// ---------------------------------------------------------------------------
// A chunk: up to 64 consecutive slots of one side of one task, or up to 64
// particles of one cell (a tile of the batched form; task = -1).
struct Chunk {
    int64_t part0;   // first particle
    int64_t slot0;   // first slot (absolute over all tasks; = part0 for tiles)
    int64_t jslot0;  // per-task: first slot of the partner side
    int32_t n;       // particles in the chunk (1..64)
    int32_t jn;      // per-task: slots of the partner side
    int32_t cell;    // origin cell (ci of the task; the tile's own cell)
    int32_t task;    // task index, -1 for a cell tile
    int32_t side;    // 0: ci side, 1: cj side
    int32_t jchunk0; // per-task: first chunk of the partner side
};
static_assert(sizeof(Chunk) == 48, "chunk layout");

// A neighbour entry of a cell: cell j and the float32 translation that moves
// j's cell-relative offsets into this cell's frame.
struct Nbr {
    int32_t cell;
    float dx, dy, dz;
};

struct CellRange {
    int64_t first;
    int32_t count;
    int32_t tile0;  // first tile of the cell
};

// One entry of a cell's flattened j-tile list: a tile of a neighbour cell,
// where its particles sit, and the float32 translation (of the neighbour
// entry) that moves its cell-relative offsets into the cell's frame.
struct JTile {
    int64_t slot0;     // first particle of the tile
    int32_t tile;      // tile index (its bounds follow the pack planes)
    int32_t n;         // particles in the tile (1..64)
    float tx, ty, tz;  // translation
    int32_t nbr;       // neighbour entry
};
static_assert(sizeof(JTile) == 32, "j-tile layout");

// lane-shuffled copy of v (DPP); rows outside ROW_MASK keep v
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

// maximum over the 64 lanes of a converged wave, returned uniform: quad swaps,
// half-row and row mirrors, then row broadcasts carry the result to lane 63
__device__ __forceinline__ float wave_max_u(float v)
{
    v = fmaxf(v, dpp<0xB1>(v));       // quad_perm [1,0,3,2]
    v = fmaxf(v, dpp<0x4E>(v));       // quad_perm [2,3,0,1]
    v = fmaxf(v, dpp<0x141>(v));      // row_half_mirror
    v = fmaxf(v, dpp<0x140>(v));      // row_mirror
    v = fmaxf(v, dpp<0x142, 0xA>(v)); // row_bcast15
    v = fmaxf(v, dpp<0x143, 0xC>(v)); // row_bcast31
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ float wave_min_u(float v)
{
    v = fminf(v, dpp<0xB1>(v));
    v = fminf(v, dpp<0x4E>(v));
    v = fminf(v, dpp<0x141>(v));
    v = fminf(v, dpp<0x140>(v));
    v = fminf(v, dpp<0x142, 0xA>(v));
    v = fminf(v, dpp<0x143, 0xC>(v));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

}  // namespace sph

struct sph_plan {
    int64_t n = 0;
    int32_t ncell = 0, ntask = 0;
    int device = 0;
    int num_cu = 256;
    std::vector<sph_cell> cells;
    std::vector<sph_task> tasks;
    std::vector<int64_t> slot_off;   // ntask + 1
    std::vector<int64_t> chunk_off;  // ntask + 1
    int64_t nslot = 0, nchunk = 0;
    int32_t ntile = 0, max_cell = 0, max_nbr = 0;
    bool batched_ok = false;
    bool mixed_widths = false;  // cells of more than one width (an octree)
    // device tables
    sph_cell *d_cells = nullptr;
    sph_task *d_tasks = nullptr;
    sph::Chunk *d_chunks = nullptr;
    sph::Chunk *d_tiles = nullptr;
    sph::CellRange *d_cellr = nullptr;
    sph::Nbr *d_nbr = nullptr;
    int32_t *d_nbr_off = nullptr;
    int32_t *d_items = nullptr;      // tiles in descending cost order
    int32_t *d_items_x = nullptr;    // per-XCD shares, each in descending cost order
    int32_t xoff[8] = {0}, xlen[8] = {0};
    int32_t *d_jt_off = nullptr;     // per cell: first entry of its j-tile list
    sph::JTile *d_jt = nullptr;      // flattened j-tiles of every cell's neighbours
    int32_t max_jt = 0;
    std::vector<int32_t> tile_off;   // per cell: its first tile (ncell + 1 entries)
    // per cell: the distance from its cube within which every non-empty cell
    // shares a task with it (a support up to this wide finds all its
    // neighbours through the cell's tasks)
    std::vector<double> reach;
    double *d_reach = nullptr;
    // copy streams of the pipelined offload step, created on its first call
    std::mutex off_mu;
    hipStream_t off_h2d = nullptr, off_d2h = nullptr;
    // per-particle slot lists, built on the first multi-task unpack
    std::mutex csr_mu;
    bool csr_built = false;
    int64_t *d_csr_off = nullptr;
    int64_t *d_csr = nullptr;
};

namespace sph {

inline int64_t round_slots(int64_t n) { return (n + 63) / 64 * 64; }

// work-queue shares of the batched form: one per XCD of the MI355X (blocks are
// dispatched to the XCDs round robin, so block b runs on XCD b mod 8); each
// share's counter sits in its own 32-byte sector of the queue area
constexpr int kQueues = 8;
constexpr int kQueueStride = 8;  // int32 counters

// floats per slot in each pack plane, per loop
constexpr int kPackPlanes[3] = {2, 3, 5};
constexpr int kPlaneFloats[3][5] = {{4, 1, 0, 0, 0}, {4, 4, 2, 0, 0}, {4, 4, 4, 4, 1}};
constexpr int kPackFloats[3] = {5, 10, 17};
constexpr int kResPlanes[3] = {3, 6, 4};
constexpr size_t kBoundsBytes = 32;  // per chunk: float4 lo {x y z Hmax}, float4 hi

// H = gamma_k h for the cubic spline (support radius over smoothing length).
constexpr float kGammaK = 1.8257418583505538f;
constexpr float kC3 = 2.5464790894703255f;  // 8 / pi

struct StoreArg {
    void *sub[kMaxSub];
};

inline StoreArg store_arg(const sph_store *s)
{
    StoreArg a;
    for (int i = 0; i < kMaxSub; ++i) a.sub[i] = s->sub[i];
    return a;
}

sph_status check_store(const sph_store *s);
sph_status check_loop(int loop);
sph_status check_range(const sph_plan *p, int32_t t0, int32_t t1);
sph_status ensure_csr(sph_plan *p);

// byte sizes of a range's buffers
inline size_t pack_bytes_for(int loop, int64_t nslot, int64_t nchunk)
{
    return (size_t)round_slots(nslot) * 4 * kPackFloats[loop] + (size_t)nchunk * kBoundsBytes;
}
inline size_t result_bytes_for(int loop, int64_t nslot)
{
    return (size_t)round_slots(nslot) * 4 * kResPlanes[loop];
}
// workspace of a batched interaction launch: the queue counter, then the
// derived per-particle planes of the gradient (1 float4) or force (2 float4 +
// 1 float2) loop
constexpr size_t kQueueBytes = 256;
// result planes of a whole staged step (every loop's outputs, in plane
// order): density 0..2, gradient 3..8, force 9..12
constexpr int kStepPlanes = 13;
constexpr int kStepPlane0[3] = {0, 3, 9};
static_assert(kQueues * kQueueStride * sizeof(int32_t) <= kQueueBytes, "queue counters");
constexpr int kDerivedFloats[3] = {0, 4, 8};
inline size_t interact_ws_bytes_for(int loop, int64_t n)
{
    return kQueueBytes + (size_t)round_slots(n) * 4 * kDerivedFloats[loop];
}

// Per-particle quantities the pair terms need beyond the packed fields: for
// the gradient loop {u, m/rho, c}; for the force loop the factors of the pair
// term with its constants folded in (see derive_force).  The batched form
// computes them once per particle into derived planes (k_prep, or the pack of
// the staged step); the per-task form computes them when it stages a
// particle.  Contraction is off inside, so every compile unit (the pack's is
// built without contraction) computes the same bits.
__device__ __forceinline__ float4 derive_gradient(const float4 &p1, const float2 &p2, float g)
{
#pragma clang fp contract(off)
    return make_float4(p2.x, p1.w / p2.y, sqrtf(g * (g - 1.0f) * p2.x), 0.f);
}

struct ForceDerived {
    float4 q0, q1;
};

// The force pair term needs, per particle, K = H^-5 (8/pi) (the spline's
// normalisation), A = P / (Omega rho^2) with P = (gamma - 1) rho u and the
// grad-h factor Omega = 1 + (h/3rho) drho/dh, the sound speed c, the
// Balsara-limited viscosity alpha~ = alpha_v |div v| / (|div v| + |curl v| +
// eps c / h), alpha_d, rho and u.  Half the spline factor w'(q)/q K is what the
// pair term uses (the average of i's and j's), and with t = 1 - q it is
//   t > 1/2:  K (9 q - 6)     = kD + nkB t,   kD = 3K, nkB = -9K
//   t <= 1/2: -3 K t^2 H / r  = kA t^2 / r,   kA = -3 K H
// (the spline is C1 at q = 1/2, so either side may take the boundary).  The
// pair sums take A2 = 2A against the halved factor, atq = -alpha~/4 and
// adh = alpha_d / 2 as the halves of the pair averages, and rh = rho / 2.
// Planes: q0 = {1/H, K, A2, c}, q1 = {atq, adh, rh, u}; kA, nkB, kD and H^2
// follow from K and h where a particle is loaded (spline_consts).
__device__ __forceinline__ ForceDerived derive_force(const float4 &p0, const float4 &p2, const float4 &p3, float ad,
                                                     float g, float eps)
{
#pragma clang fp contract(off)
    const float h = p0.w, u = p2.x, rho = p2.y, rdh = p2.z, D = p2.w;
    const float H = kGammaK * h, ih = 1.0f / H;
    const float A = (g - 1.0f) * u / (rho + h * rdh * (1.0f / 3.0f));  // P / (Omega rho^2)
    const float c = sqrtf(g * (g - 1.0f) * u);
    const float irho = 1.0f / rho;
    const float div = fabsf(D * irho);
    const float curl = sqrtf(p3.x * p3.x + p3.y * p3.y + p3.z * p3.z) * irho;
    const float at = p3.w * div / (div + curl + eps * c / h);
    const float K = kC3 * ih * ih * ih * ih * ih;
    ForceDerived f;
    f.q0 = make_float4(ih, K, 2.0f * A, c);
    f.q1 = make_float4(-0.25f * at, 0.5f * ad, 0.5f * rho, u);
    return f;
}

// ---------------------------------------------------------------------------
// launchers implemented in the .hip files
// ---------------------------------------------------------------------------
// schedule: the loop fission of sph_tuning.pack_schedule (batched form only;
// per-task ranges always use the fused kernels)
// pack of loop `loop` inside a staged step: the earlier loops' outputs are
// taken from the step's result planes (res, P floats each) instead of the
// store, and (gradient, force) the derived planes are written to `derived`
sph_status launch_pack_step(const sph_plan *p, int loop, const sph_store *s, const float *res, void *buf,
                            float *derived, const sph_params *prm, int waves, hipStream_t st);
// every output of a staged step from its result planes into the store, each
// output substruct record written whole
sph_status launch_writeback(const sph_plan *p, const sph_store *s, const float *res, int waves, hipStream_t st);
// the stage of the staged step that stores each output (1 or 2: that loop's
// pack, 3: the write-back), in step result plane order
sph_status step_writers(int layout, int32_t *writer);
sph_status launch_pack(const sph_plan *p, int loop, const sph_store *s, bool cells, int32_t t0, int32_t t1,
                       void *buf, int waves, hipStream_t st, int schedule = 0);
sph_status launch_unpack(sph_plan *p, int loop, const void *res, bool cells, int32_t t0, int32_t t1,
                         const sph_store *s, int waves, hipStream_t st, int schedule = 0);
// every member of every particle of src into dst (checked stores, same n)
sph_status launch_convert(const sph_store *src, const sph_store *dst, hipStream_t st);
// one Newton step of the smoothing-length iteration over every tile (flags[t]
// = the tile's moved particles), and the flagged tiles as a work list
sph_status launch_h_newton(const sph_plan *p, const sph_store *s, float eta, float tol, int32_t *flags,
                           hipStream_t st);
// blk: scratch of two int32 per 256 tiles; count[0] = moved particles,
// count[1] = flagged tiles
sph_status launch_flagged_tiles(const sph_plan *p, const int32_t *flags, int32_t *items, int32_t *blk,
                                int32_t *count, hipStream_t st);
// time integration: workspace of the drift / time-step reductions (the
// folded result, two doubles, at its end: integrate_ws_bytes - 256), kick,
// drift (x += v dt; result [largest distance outside a cell, largest h]) and
// the CFL step (result [unused, smallest dt])
size_t integrate_ws_bytes(const sph_plan *p);
sph_status launch_kick(const sph_store *s, float dt, hipStream_t st);
// kick: the kick by kick_dt first, in the same pass (as launch_kick, then the
// drift)
sph_status launch_drift(const sph_plan *p, const sph_store *s, double dt, void *ws, hipStream_t st,
                        bool kick = false, float kick_dt = 0.0f);
sph_status launch_cfl(const sph_plan *p, const sph_store *s, float cfl, void *ws, hipStream_t st);
// the fission groups of a layout's pack (unpack) members: bit masks as in
// sph_fission_passes, returned count (0 for an unknown layout)
int fission_passes(int layout, int loop, int schedule, bool unpack, uint32_t *masks);
sph_status launch_zero(const sph_plan *p, int loop, const sph_store *s, hipStream_t st);
// batched form over the tiles [tile0, tile1) only (the buffers keep their
// full-size layout)
sph_status launch_pack_tiles(const sph_plan *p, int loop, const sph_store *s, int32_t tile0, int32_t tile1,
                             void *buf, int waves, hipStream_t st, int schedule = 0);
sph_status launch_unpack_tiles(const sph_plan *p, int loop, const void *res, int32_t tile0, int32_t tile1,
                               const sph_store *s, int waves, hipStream_t st, int schedule = 0);
// items / nitems (batched form only): run these tiles (ascending tile order)
// instead of the plan's full list, split into per-XCD shares
sph_status launch_interact(const sph_plan *p, int loop, bool cells, int32_t t0, int32_t t1,
                           const void *pack, const sph_params *prm, const sph_tuning *tn, void *res,
                           int32_t *counts, void *ws, hipStream_t st, const int32_t *items = nullptr,
                           int64_t nitems = -1, bool prepped = false);

}  // namespace sph
