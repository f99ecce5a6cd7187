// libsph C-ABI: validation, plan construction, layout queries, store access,
// and the per-task / batched / offload entry points, the smoothing-length
// iteration and the time integration (the kernels live in sph_pack.hip,
// sph_interact.hip and sph_adjoint.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>

#include "sph_internal.hpp"

namespace sph {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }
sph_status fail(sph_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}
sph_status hip_fail(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return SPH_E_HIP;
}

static bool aligned256(const void *p) { return ((uintptr_t)p & 255u) == 0; }

sph_status check_loop(int loop)
{
    if (loop < 0 || loop > 2) return fail(SPH_E_ARG, "loop must be SPH_DENSITY, SPH_GRADIENT or SPH_FORCE");
    return SPH_OK;
}

sph_status check_store(const sph_store *s)
{
    if (!s) return fail(SPH_E_ARG, "store is null");
    if (s->layout < 0 || s->layout >= kNLayouts) return fail(SPH_E_LAYOUT, "unknown layout");
    if (s->nsub != kLayouts[s->layout].nsub)
        return fail(SPH_E_LAYOUT, "store nsub " + std::to_string(s->nsub) + " != layout's " +
                                      std::to_string(kLayouts[s->layout].nsub));
    if (s->n < 0) return fail(SPH_E_ARG, "negative particle count");
    if (s->n > 0)
        for (int i = 0; i < s->nsub; ++i) {
            if (!s->sub[i]) return fail(SPH_E_ARG, "store substruct " + std::to_string(i) + " is null");
            if (!aligned256(s->sub[i]))
                return fail(SPH_E_ARG, "store substruct " + std::to_string(i) + " is not 256-byte aligned");
        }
    return SPH_OK;
}

sph_status check_range(const sph_plan *p, int32_t t0, int32_t t1)
{
    if (t0 < 0 || t1 < t0 || t1 > p->ntask)
        return fail(SPH_E_ARG, "task range [" + std::to_string(t0) + ", " + std::to_string(t1) +
                                   ") outside [0, " + std::to_string(p->ntask) + ")");
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// generic field copy / zero (runtime descriptors; not on the hot path)
// ---------------------------------------------------------------------------
struct CompDesc {
    char *base;
    int64_t stride;
};
struct FieldDesc {
    CompDesc c[6];
    int ncomp;
    int csize;
    int nrep;                        // replicas of x written beside the primary copy
    CompDesc rep[kMaxXRep][3];
};

static FieldDesc field_desc(const sph_store *s, int f)
{
    const LayoutDesc &d = kLayouts[s->layout];
    FieldDesc fd{};
    fd.ncomp = kNComp[f];
    fd.csize = kCompBytes[f];
    for (int c = 0; c < kNComp[f]; ++c) {
        const int sb = d.sub[f][c];
        fd.c[c].base = (char *)s->sub[sb] + d.off[f][c];
        fd.c[c].stride = d.sub_bytes[sb];
    }
    fd.nrep = f == FX ? d.nxrep : 0;
    for (int r = 0; r < fd.nrep; ++r)
        for (int c = 0; c < 3; ++c) {
            const int sb = d.xrep_sub[r];
            fd.rep[r][c].base = (char *)s->sub[sb] + d.xrep_off[r] + 8 * c;
            fd.rep[r][c].stride = d.sub_bytes[sb];
        }
    return fd;
}

__global__ void k_field_copy(FieldDesc d, int64_t n, const char *src, char *dst, int to_store)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * d.ncomp) return;
    const int64_t p = i / d.ncomp;
    const int c = (int)(i - p * d.ncomp);
    char *sp = d.c[c].base + p * d.c[c].stride;
    const size_t b = (size_t)d.csize;
    if (to_store) {
        const char *q = src + i * b;
        if (b == 8) *(uint64_t *)sp = *(const uint64_t *)q;
        else if (b == 4) *(uint32_t *)sp = *(const uint32_t *)q;
        else *sp = *q;
        for (int r = 0; r < d.nrep; ++r)  // replicated positions (8-byte components)
            *(uint64_t *)(d.rep[r][c].base + p * d.rep[r][c].stride) = *(const uint64_t *)q;
    } else {
        char *q = dst + i * b;
        if (b == 8) *(uint64_t *)q = *(const uint64_t *)sp;
        else if (b == 4) *(uint32_t *)q = *(const uint32_t *)sp;
        else *q = *sp;
    }
}

__global__ void k_zero_fields(FieldDesc d, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * d.ncomp) return;
    const int64_t p = i / d.ncomp;
    const int c = (int)(i - p * d.ncomp);
    *(float *)(d.c[c].base + p * d.c[c].stride) = 0.0f;
}

// outputs of each loop (Table 1's u- columns plus the gradient loop's products)
static const int kOutField[3][6] = {{FRHO, FRHODH, FWCOUNT}, {FDIV, FROT, FROT, FROT, FLAP, FVSIG},
                                    {FA, FA, FA, FUDT}};
static const int kOutComp[3][6] = {{0, 0, 0}, {0, 0, 1, 2, 0, 0}, {0, 1, 2, 0}};

sph_status launch_zero(const sph_plan *p, int loop, const sph_store *s, hipStream_t st)
{
    (void)p;
    FieldDesc fd{};
    const LayoutDesc &d = kLayouts[s->layout];
    fd.ncomp = kResPlanes[loop];
    fd.csize = 4;
    for (int k = 0; k < fd.ncomp; ++k) {
        const int f = kOutField[loop][k], c = kOutComp[loop][k];
        const int sb = d.sub[f][c];
        fd.c[k].base = (char *)s->sub[sb] + d.off[f][c];
        fd.c[k].stride = d.sub_bytes[sb];
    }
    const int64_t tot = s->n * fd.ncomp;
    if (tot == 0) return SPH_OK;
    hipLaunchKernelGGL(k_zero_fields, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, fd, s->n);
    SPH_CHECK_LAUNCH("zero_outputs launch");
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// per-particle slot lists for multi-task unpack (host build, once per plan)
// ---------------------------------------------------------------------------
sph_status ensure_csr(sph_plan *p)
{
    std::lock_guard<std::mutex> g(p->csr_mu);
    if (p->csr_built) return SPH_OK;
    std::vector<int64_t> cnt(p->n + 1, 0);
    for (int32_t t = 0; t < p->ntask; ++t) {
        const sph_task &tk = p->tasks[t];
        const sph_cell &a = p->cells[tk.ci];
        for (int32_t k = 0; k < a.count; ++k) cnt[a.first + k + 1]++;
        if (tk.ci != tk.cj) {
            const sph_cell &b = p->cells[tk.cj];
            for (int32_t k = 0; k < b.count; ++k) cnt[b.first + k + 1]++;
        }
    }
    for (int64_t i = 0; i < p->n; ++i) cnt[i + 1] += cnt[i];
    std::vector<int64_t> lst(p->nslot), pos(cnt.begin(), cnt.end() - 1);
    int64_t slot = 0;
    for (int32_t t = 0; t < p->ntask; ++t) {
        const sph_task &tk = p->tasks[t];
        const sph_cell &a = p->cells[tk.ci];
        for (int32_t k = 0; k < a.count; ++k) lst[pos[a.first + k]++] = slot++;
        if (tk.ci != tk.cj) {
            const sph_cell &b = p->cells[tk.cj];
            for (int32_t k = 0; k < b.count; ++k) lst[pos[b.first + k]++] = slot++;
        }
    }
    SPH_HIP(hipSetDevice(p->device));
    SPH_HIP(hipMalloc(&p->d_csr_off, sizeof(int64_t) * (p->n + 1)));
    SPH_HIP(hipMalloc(&p->d_csr, sizeof(int64_t) * std::max<int64_t>(1, p->nslot)));
    SPH_HIP(hipMemcpy(p->d_csr_off, cnt.data(), sizeof(int64_t) * (p->n + 1), hipMemcpyHostToDevice));
    if (p->nslot)
        SPH_HIP(hipMemcpy(p->d_csr, lst.data(), sizeof(int64_t) * p->nslot, hipMemcpyHostToDevice));
    p->csr_built = true;
    return SPH_OK;
}

template <class T>
static sph_status upload(T **dst, const std::vector<T> &v)
{
    const size_t b = sizeof(T) * std::max<size_t>(1, v.size());
    SPH_HIP(hipMalloc((void **)dst, b));
    if (!v.empty()) SPH_HIP(hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return SPH_OK;
}

}  // namespace sph

using namespace sph;

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

const char *sph_status_str(sph_status s)
{
    switch (s) {
    case SPH_OK: return "ok";
    case SPH_E_ARG: return "invalid argument";
    case SPH_E_LAYOUT: return "layout mismatch";
    case SPH_E_CAPACITY: return "buffer too small";
    case SPH_E_PLAN: return "inconsistent plan";
    case SPH_E_HIP: return "HIP runtime error";
    case SPH_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *sph_last_error(void) { return g_err.c_str(); }

sph_status sph_layout_info(sph_layout layout, int32_t *nsub, size_t *sub_bytes)
{
    if ((int)layout < 0 || (int)layout >= kNLayouts) return fail(SPH_E_LAYOUT, "unknown layout");
    if (!nsub || !sub_bytes) return fail(SPH_E_ARG, "null output");
    const LayoutDesc &d = kLayouts[layout];
    *nsub = d.nsub;
    for (int i = 0; i < kMaxSub; ++i) sub_bytes[i] = i < d.nsub ? (size_t)d.sub_bytes[i] : 0;
    return SPH_OK;
}

sph_status sph_field_location(sph_layout layout, sph_field field, int32_t comp, int32_t *sub,
                              size_t *offset, size_t *stride)
{
    if ((int)layout < 0 || (int)layout >= kNLayouts) return fail(SPH_E_LAYOUT, "unknown layout");
    if ((int)field < 0 || (int)field >= NFIELD) return fail(SPH_E_ARG, "unknown field");
    if (comp < 0 || comp >= kNComp[field]) return fail(SPH_E_ARG, "component out of range");
    if (!sub || !offset || !stride) return fail(SPH_E_ARG, "null output");
    const LayoutDesc &d = kLayouts[layout];
    *sub = d.sub[field][comp];
    *offset = (size_t)d.off[field][comp];
    *stride = (size_t)d.sub_bytes[*sub];
    return SPH_OK;
}

sph_status sph_x_replicas(sph_layout layout, int32_t *count, int32_t *sub, size_t *offset)
{
    if ((int)layout < 0 || (int)layout >= kNLayouts) return fail(SPH_E_LAYOUT, "unknown layout");
    if (!count || !sub || !offset) return fail(SPH_E_ARG, "null output");
    const LayoutDesc &d = kLayouts[layout];
    *count = d.nxrep;
    for (int r = 0; r < d.nxrep; ++r) {
        sub[r] = d.xrep_sub[r];
        offset[r] = (size_t)d.xrep_off[r];
    }
    return SPH_OK;
}

sph_status sph_field_info(sph_field field, int32_t *ncomp, int32_t *comp_bytes)
{
    if ((int)field < 0 || (int)field >= NFIELD) return fail(SPH_E_ARG, "unknown field");
    if (!ncomp || !comp_bytes) return fail(SPH_E_ARG, "null output");
    *ncomp = kNComp[field];
    *comp_bytes = kCompBytes[field];
    return SPH_OK;
}

sph_status sph_pack_layout(sph_loop loop, int32_t *nplane, int32_t *plane_floats, int32_t *result_planes)
{
    sph_status s = check_loop(loop);
    if (s) return s;
    if (!nplane || !plane_floats || !result_planes) return fail(SPH_E_ARG, "null output");
    *nplane = kPackPlanes[loop];
    for (int k = 0; k < 5; ++k) plane_floats[k] = k < kPackPlanes[loop] ? kPlaneFloats[loop][k] : 0;
    *result_planes = kResPlanes[loop];
    return SPH_OK;
}

sph_status sph_fission_passes(sph_layout layout, sph_loop loop, int32_t schedule, int32_t *npack,
                              uint32_t *pack_masks, int32_t *nunpack, uint32_t *unpack_masks)
{
    sph_status s = check_loop(loop);
    if (s) return s;
    if ((int)layout < 0 || (int)layout >= kNLayouts) return fail(SPH_E_LAYOUT, "unknown layout");
    if (schedule < 0 || schedule > 4) return fail(SPH_E_ARG, "schedule outside 0..4");
    if (!npack || !pack_masks || !nunpack || !unpack_masks) return fail(SPH_E_ARG, "null output");
    static_assert(SPH_MAX_PASSES >= 17, "a pass per member fits");
    for (int k = 0; k < SPH_MAX_PASSES; ++k) pack_masks[k] = unpack_masks[k] = 0;
    *npack = fission_passes(layout, loop, schedule, false, pack_masks);
    *nunpack = fission_passes(layout, loop, schedule, true, unpack_masks);
    return SPH_OK;
}

static sph_status store_copy(const sph_store *store, sph_field field, const void *src, void *dst,
                             void *stream)
{
    sph_status s = check_store(store);
    if (s) return s;
    if ((int)field < 0 || (int)field >= NFIELD) return fail(SPH_E_ARG, "unknown field");
    if (store->n == 0) return SPH_OK;
    if (src == nullptr && dst == nullptr) return fail(SPH_E_ARG, "null data pointer");
    FieldDesc fd = field_desc(store, field);
    const int64_t tot = store->n * fd.ncomp;
    hipLaunchKernelGGL(k_field_copy, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, fd, store->n, (const char *)src, (char *)dst, src ? 1 : 0);
    SPH_CHECK_LAUNCH("store copy launch");
    return SPH_OK;
}

sph_status sph_store_put(const sph_store *store, sph_field field, const void *src, void *stream)
{
    if (!src) return fail(SPH_E_ARG, "src is null");
    return store_copy(store, field, src, nullptr, stream);
}

sph_status sph_store_get(const sph_store *store, sph_field field, void *dst, void *stream)
{
    if (!dst) return fail(SPH_E_ARG, "dst is null");
    return store_copy(store, field, nullptr, dst, stream);
}

sph_status sph_store_convert(const sph_store *src, const sph_store *dst, void *stream)
{
    sph_status s;
    if ((s = check_store(src)) || (s = check_store(dst))) return s;
    if (src->n != dst->n) return fail(SPH_E_ARG, "stores hold different particle counts");
    if (src->n == 0) return SPH_OK;
    // no destination substruct may share bytes with a source substruct
    for (int i = 0; i < src->nsub; ++i)
        for (int j = 0; j < dst->nsub; ++j) {
            const uintptr_t a0 = (uintptr_t)src->sub[i], a1 = a0 + (uintptr_t)src->n * kLayouts[src->layout].sub_bytes[i];
            const uintptr_t b0 = (uintptr_t)dst->sub[j], b1 = b0 + (uintptr_t)dst->n * kLayouts[dst->layout].sub_bytes[j];
            if (a0 < b1 && b0 < a1)
                return fail(SPH_E_ARG, "destination substruct " + std::to_string(j) + " overlaps source substruct " +
                                           std::to_string(i));
        }
    return launch_convert(src, dst, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
// Reach of every cell: the smallest gap (minimum image in the unit box)
// between its cube and the cube of a non-empty cell it shares no task with,
// at most 1/2.  Cells are bucketed by centre on a grid of G^3 buckets no
// narrower than the widest cell; a cell outside the 5^3 buckets around a
// cell's own is at least 1/G away from it, so the search stops there and the
// reach is at most 1/G (with G <= 5 every cell is visited).
static void compute_reach(const sph_cell *cells, int32_t nc, const sph_task *tasks, int32_t ntask,
                          std::vector<double> &reach)
{
    reach.assign(nc, 0.5);
    if (nc == 0) return;
    std::vector<int32_t> off(nc + 1, 0);
    for (int32_t t = 0; t < ntask; ++t) {
        off[tasks[t].ci + 1]++;
        if (tasks[t].cj != tasks[t].ci) off[tasks[t].cj + 1]++;
    }
    for (int32_t c = 0; c < nc; ++c) off[c + 1] += off[c];
    std::vector<int32_t> part(off[nc]);
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    for (int32_t t = 0; t < ntask; ++t) {
        part[fill[tasks[t].ci]++] = tasks[t].cj;
        if (tasks[t].cj != tasks[t].ci) part[fill[tasks[t].cj]++] = tasks[t].ci;
    }
    for (int32_t c = 0; c < nc; ++c) std::sort(part.begin() + off[c], part.begin() + off[c + 1]);
    double wmax = 0.0;
    for (int32_t c = 0; c < nc; ++c) wmax = std::max(wmax, cells[c].width);
    int64_t G = wmax > 0.0 ? (int64_t)std::floor(1.0 / wmax) : 1;
    G = std::max<int64_t>(1, std::min<int64_t>(G, 128));
    const bool all = G <= 5;
    const double cap = all ? 0.5 : std::min(0.5, 1.0 / (double)G);
    auto centre = [&](int32_t c, int d) {
        const double x = cells[c].loc[d] + 0.5 * cells[c].width;
        return x - std::floor(x);
    };
    auto bucket = [&](double x) { return std::min<int64_t>(G - 1, (int64_t)(x * (double)G)); };
    std::vector<int64_t> bstart((size_t)(G * G * G) + 1, 0);
    std::vector<int64_t> bof(nc);
    for (int32_t c = 0; c < nc; ++c) {
        bof[c] = (bucket(centre(c, 2)) * G + bucket(centre(c, 1))) * G + bucket(centre(c, 0));
        bstart[bof[c] + 1]++;
    }
    for (int64_t b = 0; b < G * G * G; ++b) bstart[b + 1] += bstart[b];
    std::vector<int32_t> bcell(nc);
    {
        std::vector<int64_t> bf(bstart.begin(), bstart.end() - 1);
        for (int32_t c = 0; c < nc; ++c) bcell[bf[bof[c]]++] = c;
    }
    auto visit = [&](int32_t c, int32_t d, double &best) {
        if (d == c || cells[d].count == 0) return;
        if (std::binary_search(part.begin() + off[c], part.begin() + off[c + 1], d)) return;
        double g2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            double dx = (cells[d].loc[k] + 0.5 * cells[d].width) - (cells[c].loc[k] + 0.5 * cells[c].width);
            dx -= std::round(dx);
            const double g = std::fabs(dx) - 0.5 * (cells[c].width + cells[d].width);
            if (g > 0.0) g2 += g * g;
        }
        best = std::min(best, std::sqrt(g2));
    };
    for (int32_t c = 0; c < nc; ++c) {
        if (cells[c].count == 0) continue;
        double best = cap;
        if (all) {
            for (int32_t d = 0; d < nc; ++d) visit(c, d, best);
        } else {
            const int64_t bx = bof[c] % G, by = (bof[c] / G) % G, bz = bof[c] / (G * G);
            for (int64_t dz = -2; dz <= 2; ++dz)
                for (int64_t dy = -2; dy <= 2; ++dy)
                    for (int64_t dx = -2; dx <= 2; ++dx) {
                        const int64_t b = (((bz + dz + G) % G) * G + (by + dy + G) % G) * G + (bx + dx + G) % G;
                        for (int64_t q = bstart[b]; q < bstart[b + 1]; ++q) visit(c, bcell[q], best);
                    }
        }
        reach[c] = best;
    }
}

sph_status sph_plan_create(const sph_cell *cells, int32_t ncell, const sph_task *tasks, int32_t ntask,
                           int64_t n, sph_plan **out)
{
    if (!out) return fail(SPH_E_ARG, "out is null");
    *out = nullptr;
    if (ncell < 0 || ntask < 0 || n < 0) return fail(SPH_E_ARG, "negative size");
    if ((ncell > 0 && !cells) || (ntask > 0 && !tasks)) return fail(SPH_E_ARG, "null cells or tasks");
    for (int32_t c = 0; c < ncell; ++c) {
        const sph_cell &e = cells[c];
        if (e.count < 0 || e.first < 0 || e.first + e.count > n)
            return fail(SPH_E_PLAN, "cell " + std::to_string(c) + " outside [0, n)");
        for (int d = 0; d < 3; ++d)
            if (!std::isfinite(e.loc[d])) return fail(SPH_E_PLAN, "cell loc not finite");
    }
    for (int32_t t = 0; t < ntask; ++t) {
        const sph_task &k = tasks[t];
        if (k.ci < 0 || k.ci >= ncell || k.cj < 0 || k.cj >= ncell)
            return fail(SPH_E_PLAN, "task " + std::to_string(t) + " names a cell out of range");
        if (k.ci == k.cj && (k.shift[0] != 0 || k.shift[1] != 0 || k.shift[2] != 0))
            return fail(SPH_E_PLAN, "self task " + std::to_string(t) + " has a shift");
        for (int d = 0; d < 3; ++d)
            if (!std::isfinite(k.shift[d])) return fail(SPH_E_PLAN, "task shift not finite");
    }

    sph_plan *p = new sph_plan();
    p->n = n;
    p->ncell = ncell;
    p->ntask = ntask;
    p->cells.assign(cells, cells + ncell);
    p->tasks.assign(tasks, tasks + ntask);
    p->slot_off.assign(ntask + 1, 0);
    p->chunk_off.assign(ntask + 1, 0);
    auto nch = [](int32_t c) { return (int64_t)((c + 63) / 64); };
    for (int32_t t = 0; t < ntask; ++t) {
        const sph_task &k = tasks[t];
        const bool pair = k.ci != k.cj;
        p->slot_off[t + 1] = p->slot_off[t] + cells[k.ci].count + (pair ? cells[k.cj].count : 0);
        p->chunk_off[t + 1] = p->chunk_off[t] + nch(cells[k.ci].count) + (pair ? nch(cells[k.cj].count) : 0);
    }
    p->nslot = p->slot_off[ntask];
    p->nchunk = p->chunk_off[ntask];
    std::vector<Chunk> ch((size_t)p->nchunk);
    for (int32_t t = 0; t < ntask; ++t) {
        const sph_task &k = tasks[t];
        const bool pair = k.ci != k.cj;
        const sph_cell &a = cells[k.ci];
        const sph_cell &b = cells[k.cj];
        int64_t ci_ch = nch(a.count);
        int64_t q = p->chunk_off[t];
        for (int64_t j = 0; j < ci_ch; ++j) {
            Chunk &c = ch[q++];
            c.part0 = a.first + 64 * j;
            c.slot0 = p->slot_off[t] + 64 * j;
            c.n = (int32_t)std::min<int64_t>(64, a.count - 64 * j);
            c.cell = k.ci;
            c.task = t;
            c.side = 0;
            c.jslot0 = pair ? p->slot_off[t] + a.count : p->slot_off[t];
            c.jn = pair ? b.count : a.count;
            c.jchunk0 = (int32_t)(pair ? p->chunk_off[t] + ci_ch : p->chunk_off[t]);
        }
        if (pair)
            for (int64_t j = 0; j < nch(b.count); ++j) {
                Chunk &c = ch[q++];
                c.part0 = b.first + 64 * j;
                c.slot0 = p->slot_off[t] + a.count + 64 * j;
                c.n = (int32_t)std::min<int64_t>(64, b.count - 64 * j);
                c.cell = k.ci;
                c.task = t;
                c.side = 1;
                c.jslot0 = p->slot_off[t];
                c.jn = a.count;
                c.jchunk0 = (int32_t)p->chunk_off[t];
            }
    }
    if (p->nchunk > INT32_MAX) {
        delete p;
        return fail(SPH_E_UNSUPPORTED, "more than 2^31 chunks");
    }

    // batched form: cells must tile the store in order
    bool ok = true;
    int64_t acc = 0;
    for (int32_t c = 0; c < ncell; ++c) {
        if (cells[c].first != acc) ok = false;
        acc += cells[c].count;
        p->max_cell = std::max(p->max_cell, cells[c].count);
    }
    if (acc != n) ok = false;
    p->batched_ok = ok;
    for (int32_t c = 1; c < ncell; ++c)
        if (cells[c].width != cells[0].width) p->mixed_widths = true;
    std::vector<Chunk> tiles;
    std::vector<CellRange> cr(ncell);
    std::vector<int32_t> nbr_off(ncell + 1, 0);
    std::vector<Nbr> nbr;
    std::vector<int32_t> items, items_x;
    std::vector<int32_t> jt_off(ncell + 1, 0);
    std::vector<JTile> jt;
    if (ok) {
        for (int32_t c = 0; c < ncell; ++c) {
            cr[c].first = cells[c].first;
            cr[c].count = cells[c].count;
            cr[c].tile0 = (int32_t)tiles.size();
            for (int32_t j = 0; j < (cells[c].count + 63) / 64; ++j) {
                Chunk t{};
                t.part0 = cells[c].first + 64 * j;
                t.slot0 = t.part0;
                t.n = std::min(64, cells[c].count - 64 * j);
                t.cell = c;
                t.task = -1;
                tiles.push_back(t);
            }
        }
        p->tile_off.resize(ncell + 1);
        for (int32_t c = 0; c < ncell; ++c) p->tile_off[c] = cr[c].tile0;
        p->tile_off[ncell] = (int32_t)tiles.size();
        std::vector<int32_t> deg(ncell, 0);
        for (const sph_task &k : p->tasks) {
            deg[k.ci]++;
            if (k.ci != k.cj) deg[k.cj]++;
        }
        for (int32_t c = 0; c < ncell; ++c) nbr_off[c + 1] = nbr_off[c] + deg[c];
        nbr.resize(nbr_off[ncell]);
        std::vector<int32_t> fillp(nbr_off.begin(), nbr_off.end() - 1);
        for (const sph_task &k : p->tasks) {
            const sph_cell &a = cells[k.ci];
            const sph_cell &b = cells[k.cj];
            if (k.ci == k.cj) {
                nbr[fillp[k.ci]++] = Nbr{k.ci, 0.f, 0.f, 0.f};
                continue;
            }
            nbr[fillp[k.ci]++] = Nbr{k.cj, (float)(b.loc[0] + k.shift[0] - a.loc[0]),
                                     (float)(b.loc[1] + k.shift[1] - a.loc[1]),
                                     (float)(b.loc[2] + k.shift[2] - a.loc[2])};
            nbr[fillp[k.cj]++] = Nbr{k.ci, (float)(a.loc[0] - k.shift[0] - b.loc[0]),
                                     (float)(a.loc[1] - k.shift[1] - b.loc[1]),
                                     (float)(a.loc[2] - k.shift[2] - b.loc[2])};
        }
        for (int32_t c = 0; c < ncell; ++c) p->max_nbr = std::max(p->max_nbr, deg[c]);
        // flattened j-tile lists: every tile of every neighbour entry, tile
        // index major (the first tile of every entry, then the second, ...), so
        // that the tiles staged into one candidate window come from all
        // directions and every lane finds a similar share of its neighbours
        // in each window
        for (int32_t c = 0; c < ncell; ++c) {
            int32_t tmax = 0;
            for (int32_t e = nbr_off[c]; e < nbr_off[c + 1]; ++e)
                tmax = std::max(tmax, (cells[nbr[e].cell].count + 63) / 64);
            for (int32_t t = 0; t < tmax; ++t) {
                for (int32_t e = nbr_off[c]; e < nbr_off[c + 1]; ++e) {
                    const int32_t nc = nbr[e].cell;
                    if (t >= (cells[nc].count + 63) / 64) continue;
                    const Chunk &tj = tiles[cr[nc].tile0 + t];
                    jt.push_back(JTile{tj.slot0, cr[nc].tile0 + t, tj.n, nbr[e].dx, nbr[e].dy, nbr[e].dz, e});
                }
            }
            jt_off[c + 1] = (int32_t)jt.size();
            p->max_jt = std::max(p->max_jt, jt_off[c + 1] - jt_off[c]);
        }
        // work items: tiles by descending candidate count (longest first)
        std::vector<int64_t> cost(tiles.size());
        for (size_t i = 0; i < tiles.size(); ++i) {
            int64_t s = 0;
            const int32_t c = tiles[i].cell;
            for (int32_t e = nbr_off[c]; e < nbr_off[c + 1]; ++e) s += cells[nbr[e].cell].count;
            cost[i] = s * tiles[i].n;
        }
        items.resize(tiles.size());
        std::iota(items.begin(), items.end(), 0);
        std::stable_sort(items.begin(), items.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
        p->ntile = (int32_t)tiles.size();
        // per-XCD shares: contiguous tile ranges (store order, so spatially
        // compact) of equal estimated cost, each in descending cost order
        items_x.resize(tiles.size());
        std::iota(items_x.begin(), items_x.end(), 0);
        int64_t total = 0;
        for (int64_t c : cost) total += c;
        int64_t run = 0;
        int32_t r = 0, start = 0;
        for (int32_t i = 0; i <= p->ntile; ++i) {
            const bool end = i == p->ntile;
            if (!end) run += cost[i];
            // close share r once it holds its fraction of the total (the last takes the rest)
            while (r < kQueues - 1 && !end && run * kQueues >= total * (r + 1)) {
                p->xoff[r] = start;
                p->xlen[r] = i + 1 - start;
                start = i + 1;
                ++r;
            }
            if (end) {
                for (; r < kQueues; ++r) {
                    p->xoff[r] = start;
                    p->xlen[r] = p->ntile - start;
                    start = p->ntile;
                }
            }
        }
        for (int32_t q = 0; q < kQueues; ++q)
            std::stable_sort(items_x.begin() + p->xoff[q], items_x.begin() + p->xoff[q] + p->xlen[q],
                             [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
    }

    compute_reach(cells, ncell, tasks, ntask, p->reach);

    sph_status st;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        delete p;
        return fail(SPH_E_HIP, "no HIP device");
    }
    p->device = dev;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
        p->num_cu = ncu;
    if ((st = upload(&p->d_cells, p->cells)) || (st = upload(&p->d_tasks, p->tasks)) ||
        (st = upload(&p->d_chunks, ch)) || (st = upload(&p->d_tiles, tiles)) || (st = upload(&p->d_cellr, cr)) ||
        (st = upload(&p->d_nbr, nbr)) || (st = upload(&p->d_nbr_off, nbr_off)) || (st = upload(&p->d_items, items)) || (st = upload(&p->d_items_x, items_x)) ||
        (st = upload(&p->d_jt_off, jt_off)) || (st = upload(&p->d_jt, jt)) || (st = upload(&p->d_reach, p->reach))) {
        sph_plan_destroy(p);
        return st;
    }
    *out = p;
    return SPH_OK;
}

void sph_plan_destroy(sph_plan *p)
{
    if (!p) return;
    (void)hipSetDevice(p->device);
    void *ptrs[] = {p->d_cells, p->d_tasks, p->d_chunks, p->d_tiles, p->d_cellr, p->d_nbr,
                    p->d_nbr_off, p->d_items, p->d_items_x, p->d_jt_off, p->d_jt, p->d_csr_off, p->d_csr,
                    p->d_reach};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    if (p->off_h2d) (void)hipStreamDestroy(p->off_h2d);
    if (p->off_d2h) (void)hipStreamDestroy(p->off_d2h);
    delete p;
}

sph_status sph_plan_get_info(const sph_plan *p, sph_plan_info *info)
{
    if (!p || !info) return fail(SPH_E_ARG, "null argument");
    info->n = p->n;
    info->ncell = p->ncell;
    info->ntask = p->ntask;
    info->nslot = p->nslot;
    info->nchunk = p->nchunk;
    info->ntile = p->ntile;
    info->max_cell = p->max_cell;
    info->max_nbr = p->max_nbr;
    info->batched_ok = p->batched_ok ? 1 : 0;
    info->mixed_widths = p->mixed_widths ? 1 : 0;
    info->pad = 0;
    return SPH_OK;
}

sph_status sph_plan_cell_reach(const sph_plan *p, double *reach)
{
    if (!p || (!reach && p->ncell > 0)) return fail(SPH_E_ARG, "null argument");
    std::copy(p->reach.begin(), p->reach.end(), reach);
    return SPH_OK;
}

sph_status sph_plan_buffer_bytes(const sph_plan *p, sph_loop loop, int32_t t0, int32_t t1, int64_t *nslot,
                                 size_t *pack_bytes, size_t *result_bytes)
{
    if (!p) return fail(SPH_E_ARG, "plan is null");
    sph_status s;
    if ((s = check_loop(loop)) || (s = check_range(p, t0, t1))) return s;
    const int64_t ns = p->slot_off[t1] - p->slot_off[t0];
    const int64_t nc = p->chunk_off[t1] - p->chunk_off[t0];
    if (nslot) *nslot = ns;
    if (pack_bytes) *pack_bytes = pack_bytes_for(loop, ns, nc);
    if (result_bytes) *result_bytes = result_bytes_for(loop, ns);
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// per-task / bundled path
// ---------------------------------------------------------------------------
sph_status sph_zero_outputs(const sph_plan *p, sph_loop loop, const sph_store *store, void *stream)
{
    if (!p) return fail(SPH_E_ARG, "plan is null");
    sph_status s;
    if ((s = check_loop(loop)) || (s = check_store(store))) return s;
    if (store->n != p->n) return fail(SPH_E_ARG, "store size differs from the plan's");
    return launch_zero(p, loop, store, (hipStream_t)stream);
}

sph_status sph_pack(const sph_plan *p, sph_loop loop, const sph_store *store, int32_t t0, int32_t t1,
                    void *pack_buf, size_t pack_bytes, void *stream)
{
    if (!p) return fail(SPH_E_ARG, "plan is null");
    sph_status s;
    if ((s = check_loop(loop)) || (s = check_store(store)) || (s = check_range(p, t0, t1))) return s;
    if (store->n != p->n) return fail(SPH_E_ARG, "store size differs from the plan's");
    const int64_t ns = p->slot_off[t1] - p->slot_off[t0];
    if (ns == 0) return SPH_OK;
    const size_t need = pack_bytes_for(loop, ns, p->chunk_off[t1] - p->chunk_off[t0]);
    if (!pack_buf) return fail(SPH_E_ARG, "pack buffer is null");
    if (!aligned256(pack_buf)) return fail(SPH_E_ARG, "pack buffer is not 256-byte aligned");
    if (pack_bytes < need) return fail(SPH_E_CAPACITY, "pack buffer needs " + std::to_string(need) + " bytes");
    return launch_pack(p, loop, store, false, t0, t1, pack_buf, 4, (hipStream_t)stream);
}

static sph_status interact_checked(const sph_plan *p, int loop, const void *pack_buf, size_t pack_bytes,
                                   int32_t t0, int32_t t1, const sph_params *prm, void *res_buf,
                                   size_t res_bytes, int32_t *counts, void *stream)
{
    if (!p) return fail(SPH_E_ARG, "plan is null");
    sph_status s;
    if ((s = check_range(p, t0, t1))) return s;
    if (!prm) return fail(SPH_E_ARG, "params is null");
    const int64_t ns = p->slot_off[t1] - p->slot_off[t0];
    if (ns == 0) return SPH_OK;
    if (!pack_buf || !res_buf) return fail(SPH_E_ARG, "null buffer");
    if (!aligned256(pack_buf) || !aligned256(res_buf)) return fail(SPH_E_ARG, "buffer not 256-byte aligned");
    if (pack_bytes < pack_bytes_for(loop, ns, p->chunk_off[t1] - p->chunk_off[t0]))
        return fail(SPH_E_CAPACITY, "pack buffer too small for the range");
    if (res_bytes < result_bytes_for(loop, ns)) return fail(SPH_E_CAPACITY, "result buffer too small");
    return launch_interact(p, loop, false, t0, t1, pack_buf, prm, nullptr, res_buf, counts, nullptr,
                           (hipStream_t)stream);
}

sph_status sph_density(const sph_plan *p, const void *pack_buf, size_t pack_bytes, int32_t t0, int32_t t1,
                       const sph_params *prm, void *res_buf, size_t res_bytes, int32_t *counts, void *stream)
{
    return interact_checked(p, 0, pack_buf, pack_bytes, t0, t1, prm, res_buf, res_bytes, counts, stream);
}
sph_status sph_gradient(const sph_plan *p, const void *pack_buf, size_t pack_bytes, int32_t t0, int32_t t1,
                        const sph_params *prm, void *res_buf, size_t res_bytes, int32_t *counts, void *stream)
{
    return interact_checked(p, 1, pack_buf, pack_bytes, t0, t1, prm, res_buf, res_bytes, counts, stream);
}
sph_status sph_force(const sph_plan *p, const void *pack_buf, size_t pack_bytes, int32_t t0, int32_t t1,
                     const sph_params *prm, void *res_buf, size_t res_bytes, int32_t *counts, void *stream)
{
    return interact_checked(p, 2, pack_buf, pack_bytes, t0, t1, prm, res_buf, res_bytes, counts, stream);
}

sph_status sph_unpack(const sph_plan *p, sph_loop loop, const void *res_buf, size_t res_bytes, int32_t t0,
                      int32_t t1, const sph_store *store, void *stream)
{
    if (!p) return fail(SPH_E_ARG, "plan is null");
    sph_status s;
    if ((s = check_loop(loop)) || (s = check_store(store)) || (s = check_range(p, t0, t1))) return s;
    if (store->n != p->n) return fail(SPH_E_ARG, "store size differs from the plan's");
    const int64_t ns = p->slot_off[t1] - p->slot_off[t0];
    if (ns == 0) return SPH_OK;
    if (!res_buf) return fail(SPH_E_ARG, "result buffer is null");
    if (!aligned256(res_buf)) return fail(SPH_E_ARG, "result buffer not 256-byte aligned");
    if (res_bytes < result_bytes_for(loop, ns)) return fail(SPH_E_CAPACITY, "result buffer too small");
    sph_plan *mp = const_cast<sph_plan *>(p);
    if (t1 - t0 > 1 && (s = ensure_csr(mp))) return s;
    return launch_unpack(mp, loop, res_buf, false, t0, t1, store, 4, (hipStream_t)stream);
}

sph_status sph_plan_task_max_bytes(const sph_plan *p, sph_loop loop, size_t *pack_bytes, size_t *result_bytes)
{
    if (!p || !pack_bytes || !result_bytes) return fail(SPH_E_ARG, "null argument");
    sph_status s;
    if ((s = check_loop(loop))) return s;
    size_t pb = 0, rb = 0;
    for (int32_t t = 0; t < p->ntask; ++t) {
        const int64_t ns = p->slot_off[t + 1] - p->slot_off[t];
        const int64_t nc = p->chunk_off[t + 1] - p->chunk_off[t];
        pb = std::max(pb, pack_bytes_for(loop, ns, nc));
        rb = std::max(rb, result_bytes_for(loop, ns));
    }
    *pack_bytes = pb;
    *result_bytes = rb;
    return SPH_OK;
}

sph_status sph_run_per_task(const sph_plan *p, sph_loop loop, const sph_store *store, int32_t t0, int32_t t1,
                            int32_t zero_first, const sph_params *prm, void *pack_buf, size_t pack_bytes,
                            void *res_buf, size_t res_bytes, void *stream)
{
    if (!p) return fail(SPH_E_ARG, "plan is null");
    sph_status s;
    if ((s = check_loop(loop)) || (s = check_store(store)) || (s = check_range(p, t0, t1))) return s;
    if (!prm) return fail(SPH_E_ARG, "params is null");
    if (store->n != p->n) return fail(SPH_E_ARG, "store size differs from the plan's");
    if (!pack_buf || !res_buf || !aligned256(pack_buf) || !aligned256(res_buf))
        return fail(SPH_E_ARG, "buffer null or not 256-byte aligned");
    for (int32_t t = t0; t < t1; ++t) {
        const int64_t ns = p->slot_off[t + 1] - p->slot_off[t];
        if (pack_bytes < pack_bytes_for(loop, ns, p->chunk_off[t + 1] - p->chunk_off[t]) ||
            res_bytes < result_bytes_for(loop, ns))
            return fail(SPH_E_CAPACITY, "buffers smaller than task " + std::to_string(t));
    }
    hipStream_t st = (hipStream_t)stream;
    if (zero_first && (s = launch_zero(p, loop, store, st))) return s;
    sph_plan *mp = const_cast<sph_plan *>(p);
    for (int32_t t = t0; t < t1; ++t) {
        if (p->slot_off[t + 1] == p->slot_off[t]) continue;
        if ((s = launch_pack(p, loop, store, false, t, t + 1, pack_buf, 4, st))) return s;
        if ((s = launch_interact(p, loop, false, t, t + 1, pack_buf, prm, nullptr, res_buf, nullptr, nullptr, st)))
            return s;
        if ((s = launch_unpack(mp, loop, res_buf, false, t, t + 1, store, 4, st))) return s;
    }
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// batched form
// ---------------------------------------------------------------------------
void sph_tuning_default(sph_tuning *t)
{
    if (!t) return;
    std::memset(t, 0, sizeof(*t));
    t->blocks_per_cu = 8;
    t->window[0] = 256;
    t->window[1] = 256;
    t->window[2] = 128;
    t->pack_waves = 4;
    t->queue = 1;
}

static sph_status check_tuning(const sph_tuning *t)
{
    if (!t) return SPH_OK;
    if (t->blocks_per_cu < 1 || t->blocks_per_cu > 64) return fail(SPH_E_ARG, "blocks_per_cu outside 1..64");
    for (int k = 0; k < 3; ++k)
        if (t->window[k] != 128 && t->window[k] != 256 && t->window[k] != 512)
            return fail(SPH_E_ARG, "window must be 128, 256 or 512");
    if (t->pack_waves < 1 || t->pack_waves > 8) return fail(SPH_E_ARG, "pack_waves outside 1..8");
    if (t->queue < 0 || t->queue > 2) return fail(SPH_E_ARG, "queue must be 0, 1 or 2");
    if (t->pack_schedule < 0 || t->pack_schedule > 4) return fail(SPH_E_ARG, "pack_schedule outside 0..4");
    for (int k = 0; k < 3; ++k)
        if (t->blocks_per_loop[k] < 0 || t->blocks_per_loop[k] > 64)
            return fail(SPH_E_ARG, "blocks_per_loop outside 0..64");
    return SPH_OK;
}

static sph_status batched_checks(const sph_plan *p, int loop)
{
    if (!p) return fail(SPH_E_ARG, "plan is null");
    sph_status s;
    if ((s = check_loop(loop))) return s;
    if (!p->batched_ok) return fail(SPH_E_UNSUPPORTED, "cells do not tile the store in order");
    return SPH_OK;
}

// workspace of the staged step: the interaction workspace (queue counters and
// derived planes) of the force loop, the largest pack buffer, then the result
// planes of all three loops
struct StepWs {
    char *q;      // interaction workspace
    char *pack;   // pack buffer
    float *res;   // kStepPlanes planes of round_slots(n) floats
};
static size_t step_ws_bytes(const sph_plan *p)
{
    return interact_ws_bytes_for(2, p->n) + pack_bytes_for(2, p->n, p->ntile) +
           (size_t)round_slots(p->n) * 4 * kStepPlanes;
}
static StepWs step_ws(const sph_plan *p, void *ws)
{
    StepWs w;
    w.q = (char *)ws;
    w.pack = w.q + interact_ws_bytes_for(2, p->n);
    w.res = (float *)(w.pack + pack_bytes_for(2, p->n, p->ntile));
    return w;
}

sph_status sph_batched_ws_bytes(const sph_plan *p, size_t *bytes)
{
    if (!p || !bytes) return fail(SPH_E_ARG, "null argument");
    *bytes = step_ws_bytes(p);
    return SPH_OK;
}

sph_status sph_interact_ws_bytes(const sph_plan *p, sph_loop loop, size_t *bytes)
{
    if (!p || !bytes) return fail(SPH_E_ARG, "null argument");
    sph_status s;
    if ((s = check_loop(loop))) return s;
    *bytes = interact_ws_bytes_for(loop, p->n);
    return SPH_OK;
}

sph_status sph_pack_cells(const sph_plan *p, sph_loop loop, const sph_store *store, void *pack_buf,
                          size_t pack_bytes, const sph_tuning *tn, void *stream)
{
    sph_status s;
    if ((s = batched_checks(p, loop)) || (s = check_store(store)) || (s = check_tuning(tn))) return s;
    if (store->n != p->n) return fail(SPH_E_ARG, "store size differs from the plan's");
    if (p->n == 0) return SPH_OK;
    if (!pack_buf || !aligned256(pack_buf)) return fail(SPH_E_ARG, "pack buffer null or misaligned");
    if (pack_bytes < pack_bytes_for(loop, p->n, p->ntile)) return fail(SPH_E_CAPACITY, "pack buffer too small");
    return launch_pack(p, loop, store, true, 0, 0, pack_buf, tn ? tn->pack_waves : 4, (hipStream_t)stream,
                       tn ? tn->pack_schedule : 0);
}

sph_status sph_interact_cells(const sph_plan *p, sph_loop loop, const void *pack_buf, size_t pack_bytes,
                              const sph_params *prm, const sph_tuning *tn, void *res_buf, size_t res_bytes,
                              int32_t *counts, void *ws, size_t ws_bytes, void *stream)
{
    sph_status s;
    if ((s = batched_checks(p, loop)) || (s = check_tuning(tn))) return s;
    if (!prm) return fail(SPH_E_ARG, "params is null");
    if (p->n == 0) return SPH_OK;
    if (!pack_buf || !res_buf || !ws) return fail(SPH_E_ARG, "null buffer or workspace");
    if (ws_bytes < interact_ws_bytes_for(loop, p->n))
        return fail(SPH_E_CAPACITY, "workspace needs " + std::to_string(interact_ws_bytes_for(loop, p->n)) + " bytes");
    if (!aligned256(pack_buf) || !aligned256(res_buf) || !aligned256(ws))
        return fail(SPH_E_ARG, "buffer not 256-byte aligned");
    if (pack_bytes < pack_bytes_for(loop, p->n, p->ntile)) return fail(SPH_E_CAPACITY, "pack buffer too small");
    if (res_bytes < result_bytes_for(loop, p->n)) return fail(SPH_E_CAPACITY, "result buffer too small");
    sph_tuning def;
    sph_tuning_default(&def);
    return launch_interact(p, loop, true, 0, p->ntask, pack_buf, prm, tn ? tn : &def, res_buf, counts, ws,
                           (hipStream_t)stream);
}

sph_status sph_unpack_cells(const sph_plan *p, sph_loop loop, const void *res_buf, size_t res_bytes,
                            const sph_store *store, const sph_tuning *tn, void *stream)
{
    sph_status s;
    if ((s = batched_checks(p, loop)) || (s = check_store(store)) || (s = check_tuning(tn))) return s;
    if (store->n != p->n) return fail(SPH_E_ARG, "store size differs from the plan's");
    if (p->n == 0) return SPH_OK;
    if (!res_buf || !aligned256(res_buf)) return fail(SPH_E_ARG, "result buffer null or misaligned");
    if (res_bytes < result_bytes_for(loop, p->n)) return fail(SPH_E_CAPACITY, "result buffer too small");
    return launch_unpack(const_cast<sph_plan *>(p), loop, res_buf, true, 0, 0, store, tn ? tn->pack_waves : 4,
                         (hipStream_t)stream, tn ? tn->pack_schedule : 0);
}

static sph_status step_batched(const sph_plan *p, const sph_store *store, const sph_params *prm,
                               const sph_tuning *tn, void *ws, size_t ws_bytes, hipStream_t st)
{
    sph_status s;
    if ((s = batched_checks(p, 0)) || (s = check_store(store)) || (s = check_tuning(tn))) return s;
    if (!prm) return fail(SPH_E_ARG, "params is null");
    if (store->n != p->n) return fail(SPH_E_ARG, "store size differs from the plan's");
    size_t need = 0;
    sph_batched_ws_bytes(p, &need);
    if (!ws || !aligned256(ws)) return fail(SPH_E_ARG, "workspace null or misaligned");
    if (ws_bytes < need) return fail(SPH_E_CAPACITY, "workspace needs " + std::to_string(need) + " bytes");
    if (p->n == 0) return SPH_OK;
    sph_tuning def;
    sph_tuning_default(&def);
    if (!tn) tn = &def;
    const StepWs w = step_ws(p, ws);
    if (tn->pack_schedule != 0) {
        // loop-fission schedules: each loop's own unpack into the store, then
        // the next loop packs from it
        for (int loop = 0; loop < 3; ++loop) {
            if ((s = launch_pack(p, loop, store, true, 0, 0, w.pack, tn->pack_waves, st, tn->pack_schedule)))
                return s;
            if ((s = launch_interact(p, loop, true, 0, p->ntask, w.pack, prm, tn, w.res, nullptr, w.q, st)))
                return s;
            if ((s = launch_unpack(const_cast<sph_plan *>(p), loop, w.res, true, 0, 0, store, tn->pack_waves, st,
                                   tn->pack_schedule)))
                return s;
        }
        return SPH_OK;
    }
    // staged: outputs stay in the step's result planes, later packs read them
    // there, and one write-back stores them all
    for (int loop = 0; loop < 3; ++loop) {
        if ((s = launch_pack_step(p, loop, store, w.res, w.pack, (float *)(w.q + kQueueBytes), prm, tn->pack_waves,
                                  st)))
            return s;
        if ((s = launch_interact(p, loop, true, 0, p->ntask, w.pack, prm, tn,
                                 w.res + (size_t)kStepPlane0[loop] * round_slots(p->n), nullptr, w.q, st, nullptr,
                                 -1, true)))
            return s;
    }
    return launch_writeback(p, store, w.res, tn->pack_waves, st);
}

static sph_status step_stage_checks(const sph_plan *p, const sph_store *store, const sph_tuning *tn, void *ws,
                                    size_t ws_bytes)
{
    sph_status s;
    if ((s = batched_checks(p, 0)) || (store && (s = check_store(store))) || (s = check_tuning(tn))) return s;
    if (store && store->n != p->n) return fail(SPH_E_ARG, "store size differs from the plan's");
    if (!ws || !aligned256(ws)) return fail(SPH_E_ARG, "workspace null or misaligned");
    if (ws_bytes < step_ws_bytes(p))
        return fail(SPH_E_CAPACITY, "workspace needs " + std::to_string(step_ws_bytes(p)) + " bytes");
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// allocation-free batched step: the workspace lives in a file-scope device
// array, one copy per GPU the library runs on, held until the process ends
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[SPH_NOALLOC_SCRATCH_BYTES];

// device address of this GPU's copy of `scratch`, looked up once per device
// with that device current (in host code the array's name is not a device
// address)
static sph_status scratch_address(void **out)
{
    constexpr int kMaxDev = 64;
    static void *addr[kMaxDev] = {};
    static std::mutex mu;
    int dev = -1;
    SPH_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) return fail(SPH_E_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(SPH_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        addr[dev] = ptr;
    }
    *out = addr[dev];
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// smoothing-length iteration
// ---------------------------------------------------------------------------
static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// workspace: interaction workspace, pack and result buffers of the density
// loop, tile flags, tile work list, per-256-tile counts, two counters
static size_t h_iter_ws_bytes_for(const sph_plan *p)
{
    return interact_ws_bytes_for(0, p->n) + align256(pack_bytes_for(0, p->n, p->ntile)) +
           align256(result_bytes_for(0, p->n)) + 2 * align256((size_t)p->ntile * 4) +
           align256(((size_t)p->ntile + 255) / 256 * 8) + 256;
}

sph_status sph_h_iterate_ws_bytes(const sph_plan *p, size_t *bytes)
{
    if (!p || !bytes) return fail(SPH_E_ARG, "null argument");
    *bytes = h_iter_ws_bytes_for(p);
    return SPH_OK;
}

sph_status sph_h_iterate(const sph_plan *p, const sph_store *store, const sph_params *prm, const sph_tuning *tn,
                         float eta, float tol, int32_t max_iter, void *ws, size_t ws_bytes, int32_t *iterations,
                         int64_t *unconverged, void *stream)
{
    sph_status s;
    if ((s = batched_checks(p, 0)) || (s = check_store(store)) || (s = check_tuning(tn))) return s;
    if (!prm) return fail(SPH_E_ARG, "params is null");
    if (store->n != p->n) return fail(SPH_E_ARG, "store size differs from the plan's");
    if (!(eta > 0.0f) || !(tol > 0.0f) || max_iter < 1)
        return fail(SPH_E_ARG, "eta and tol must be positive and max_iter at least 1");
    if (!ws || !aligned256(ws)) return fail(SPH_E_ARG, "workspace null or misaligned");
    if (ws_bytes < h_iter_ws_bytes_for(p))
        return fail(SPH_E_CAPACITY, "workspace needs " + std::to_string(h_iter_ws_bytes_for(p)) + " bytes");
    if (iterations) *iterations = 0;
    if (unconverged) *unconverged = 0;
    if (p->n == 0) return SPH_OK;
    sph_tuning def;
    sph_tuning_default(&def);
    if (!tn) tn = &def;
    const hipStream_t st = (hipStream_t)stream;
    char *base = (char *)ws;
    void *q = base;
    char *pack = base + interact_ws_bytes_for(0, p->n);
    char *res = pack + align256(pack_bytes_for(0, p->n, p->ntile));
    int32_t *flags = (int32_t *)(res + align256(result_bytes_for(0, p->n)));
    int32_t *items = (int32_t *)((char *)flags + align256((size_t)p->ntile * 4));
    int32_t *blk = (int32_t *)((char *)items + align256((size_t)p->ntile * 4));
    int32_t *cnt = (int32_t *)((char *)blk + align256(((size_t)p->ntile + 255) / 256 * 8));  // [0] moved, [1] tiles
    int64_t nitems = -1;  // the first pass runs every tile
    int32_t host_cnt[2] = {0, 0};
    for (int it = 0; it < max_iter; ++it) {
        if ((s = launch_pack(p, 0, store, true, 0, 0, pack, tn->pack_waves, st, tn->pack_schedule))) return s;
        if ((s = launch_interact(p, 0, true, 0, p->ntask, pack, prm, tn, res, nullptr, q, st,
                                 nitems < 0 ? nullptr : items, nitems)))
            return s;
        if ((s = launch_unpack(const_cast<sph_plan *>(p), 0, res, true, 0, 0, store, tn->pack_waves, st,
                               tn->pack_schedule)))
            return s;
        if ((s = launch_h_newton(p, store, eta, tol, flags, st))) return s;
        if ((s = launch_flagged_tiles(p, flags, items, blk, cnt, st))) return s;
        SPH_HIP(hipMemcpyAsync(host_cnt, cnt, sizeof(host_cnt), hipMemcpyDeviceToHost, st));
        SPH_HIP(hipStreamSynchronize(st));
        if (iterations) *iterations = it + 1;
        if (unconverged) *unconverged = host_cnt[0];
        if (host_cnt[0] == 0) break;
        nitems = host_cnt[1];
    }
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// time integration around the loops
// ---------------------------------------------------------------------------
sph_status sph_integrate_ws_bytes(const sph_plan *p, size_t *bytes)
{
    if (!p || !bytes) return fail(SPH_E_ARG, "null argument");
    *bytes = integrate_ws_bytes(p);
    return SPH_OK;
}

sph_status sph_kick(const sph_store *store, float dt, void *stream)
{
    sph_status s = check_store(store);
    if (s) return s;
    if (!std::isfinite(dt)) return fail(SPH_E_ARG, "dt is not finite");
    return launch_kick(store, dt, (hipStream_t)stream);
}

static sph_status integrate_checks(const sph_plan *p, const sph_store *store, void *ws, size_t ws_bytes)
{
    sph_status s;
    if ((s = batched_checks(p, 0)) || (s = check_store(store))) return s;
    if (store->n != p->n) return fail(SPH_E_ARG, "store size differs from the plan's");
    if (!ws || !aligned256(ws)) return fail(SPH_E_ARG, "workspace null or misaligned");
    if (ws_bytes < integrate_ws_bytes(p))
        return fail(SPH_E_CAPACITY, "workspace needs " + std::to_string(integrate_ws_bytes(p)) + " bytes");
    return SPH_OK;
}

// the folded reduction result at the end of the workspace, copied to the host
static sph_status read_fold(const sph_plan *p, void *ws, double out[2], hipStream_t st)
{
    const char *r = (const char *)ws + integrate_ws_bytes(p) - 256;
    SPH_HIP(hipMemcpyAsync(out, r, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    SPH_HIP(hipStreamSynchronize(st));
    return SPH_OK;
}

sph_status sph_drift(const sph_plan *p, const sph_store *store, double dt, void *ws, size_t ws_bytes,
                     double *max_outside, float *max_h, void *stream)
{
    sph_status s;
    if ((s = integrate_checks(p, store, ws, ws_bytes))) return s;
    if (!std::isfinite(dt)) return fail(SPH_E_ARG, "dt is not finite");
    if (p->n == 0) {
        if (max_outside) *max_outside = 0.0;
        if (max_h) *max_h = 0.0f;
        return SPH_OK;
    }
    if ((s = launch_drift(p, store, dt, ws, (hipStream_t)stream))) return s;
    if (max_outside || max_h) {
        double r[2];
        if ((s = read_fold(p, ws, r, (hipStream_t)stream))) return s;
        if (max_outside) *max_outside = r[0];
        if (max_h) *max_h = (float)r[1];
    }
    return SPH_OK;
}

sph_status sph_cfl_dt(const sph_plan *p, const sph_store *store, float cfl, void *ws, size_t ws_bytes, float *dt,
                      void *stream)
{
    sph_status s;
    if ((s = integrate_checks(p, store, ws, ws_bytes))) return s;
    if (!(cfl > 0.0f) || !dt) return fail(SPH_E_ARG, "cfl must be positive and dt non-null");
    *dt = __builtin_huge_valf();
    if (p->n == 0) return SPH_OK;
    if ((s = launch_cfl(p, store, cfl, ws, (hipStream_t)stream))) return s;
    double r[2];
    if ((s = read_fold(p, ws, r, (hipStream_t)stream))) return s;
    *dt = (float)r[1];
    return SPH_OK;
}

sph_status sph_step_kdk(const sph_plan *p, const sph_store *store, const sph_params *prm, const sph_tuning *tn,
                        float dt, void *ws, size_t ws_bytes, int32_t *rebuild, void *stream)
{
    sph_status s;
    size_t step_bytes = 0;
    sph_batched_ws_bytes(p, &step_bytes);
    step_bytes = (step_bytes + 255) / 256 * 256;
    if (!p) return fail(SPH_E_ARG, "plan is null");
    if (ws_bytes < step_bytes) return fail(SPH_E_CAPACITY, "workspace too small");
    if ((s = integrate_checks(p, store, (char *)ws + step_bytes, ws_bytes - step_bytes))) return s;
    if (!prm) return fail(SPH_E_ARG, "params is null");
    if (!std::isfinite(dt) || !(dt >= 0.0f)) return fail(SPH_E_ARG, "dt must be finite and non-negative");
    if (rebuild) *rebuild = 0;
    if (p->n == 0) return SPH_OK;
    const hipStream_t st = (hipStream_t)stream;
    void *iws = (char *)ws + step_bytes;
    const float half = 0.5f * dt;
    // the first half kick and the drift in one pass over the particles
    if ((s = launch_drift(p, store, (double)dt, iws, st, true, half))) return s;
    double r[2];
    if ((s = read_fold(p, iws, r, st))) return s;
    // every pair within a support must still meet in cells that share a task:
    // H_max + 2 (largest distance outside a cell) <= the smallest reach
    double wmin = __builtin_huge_val();
    for (int32_t c = 0; c < p->ncell; ++c)
        if (p->cells[c].count > 0) wmin = std::min(wmin, p->reach[c]);
    if ((double)kGammaK * r[1] + 2.0 * r[0] > wmin) {
        if (rebuild) *rebuild = 1;
        return fail(SPH_E_PLAN, "particles drifted beyond the plan's reach: rebuild the plan, then run the "
                                "loops and the second half kick");
    }
    if ((s = step_batched(p, store, prm, tn, ws, step_bytes, st))) return s;
    return launch_kick(store, half, st);
}

sph_status sph_step_batched(const sph_plan *p, const sph_store *store, const sph_params *prm,
                            const sph_tuning *tn, void *ws, size_t ws_bytes, void *stream)
{
    return step_batched(p, store, prm, tn, ws, ws_bytes, (hipStream_t)stream);
}

sph_status sph_step_pack(const sph_plan *p, sph_loop loop, const sph_store *store, const sph_params *prm,
                         const sph_tuning *tn, void *ws, size_t ws_bytes, void *stream)
{
    sph_status s;
    if ((s = check_loop(loop)) || (s = step_stage_checks(p, store, tn, ws, ws_bytes))) return s;
    if (!prm) return fail(SPH_E_ARG, "params is null");
    if (p->n == 0) return SPH_OK;
    const StepWs w = step_ws(p, ws);
    return launch_pack_step(p, loop, store, w.res, w.pack, (float *)(w.q + kQueueBytes), prm, tn ? tn->pack_waves : 4,
                            (hipStream_t)stream);
}

sph_status sph_step_interact(const sph_plan *p, sph_loop loop, const sph_params *prm, const sph_tuning *tn,
                             void *ws, size_t ws_bytes, void *stream)
{
    sph_status s;
    if ((s = check_loop(loop)) || (s = step_stage_checks(p, nullptr, tn, ws, ws_bytes))) return s;
    if (!prm) return fail(SPH_E_ARG, "params is null");
    if (p->n == 0) return SPH_OK;
    sph_tuning def;
    sph_tuning_default(&def);
    const StepWs w = step_ws(p, ws);
    return launch_interact(p, loop, true, 0, p->ntask, w.pack, prm, tn ? tn : &def,
                           w.res + (size_t)kStepPlane0[loop] * round_slots(p->n), nullptr, w.q, (hipStream_t)stream,
                           nullptr, -1, true);
}

sph_status sph_step_output_writers(sph_layout layout, int32_t *writer)
{
    if ((int)layout < 0 || (int)layout >= kNLayouts) return fail(SPH_E_LAYOUT, "unknown layout");
    if (!writer) return fail(SPH_E_ARG, "null output");
    return step_writers((int)layout, writer);
}

sph_status sph_step_writeback(const sph_plan *p, const sph_store *store, const sph_tuning *tn, void *ws,
                              size_t ws_bytes, void *stream)
{
    sph_status s;
    if ((s = step_stage_checks(p, store, tn, ws, ws_bytes))) return s;
    if (!store) return fail(SPH_E_ARG, "store is null");
    if (p->n == 0) return SPH_OK;
    return launch_writeback(p, store, step_ws(p, ws).res, tn ? tn->pack_waves : 4, (hipStream_t)stream);
}

sph_status sph_step_batched_noalloc(const sph_plan *p, const sph_store *store, const sph_params *prm,
                                    const sph_tuning *tn, void *stream)
{
    if (!p) return fail(SPH_E_ARG, "plan is null");
    size_t need = 0;
    sph_batched_ws_bytes(p, &need);
    if (need > (size_t)SPH_NOALLOC_SCRATCH_BYTES)
        return fail(SPH_E_CAPACITY, "the step needs " + std::to_string(need) + " bytes of workspace, beyond the " +
                                        std::to_string((size_t)SPH_NOALLOC_SCRATCH_BYTES) +
                                        "-byte static scratch: use sph_step_batched with a workspace");
    void *ws = nullptr;
    sph_status s = scratch_address(&ws);
    if (s) return s;
    return step_batched(p, store, prm, tn, ws, (size_t)SPH_NOALLOC_SCRATCH_BYTES, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// offload form
// ---------------------------------------------------------------------------
// fields each loop's pack reads (Table 1, extended as for the pack records)
static const int kReadFields[3][11] = {{FX, FMASS, FH, -1},
                                       {FX, FV, FMASS, FH, FU, FRHO, -1},
                                       {FX, FV, FMASS, FH, FU, FRHO, FRHODH, FDIV, FROT, FAV, FAD}};

static bool loop_reads(int loop, int f)
{
    for (int k = 0; k < 11 && kReadFields[loop][k] >= 0; ++k)
        if (kReadFields[loop][k] == f) return true;
    return false;
}
static bool loop_writes(int loop, int f)
{
    for (int k = 0; k < kResPlanes[loop]; ++k)
        if (kOutField[loop][k] == f) return true;
    return false;
}

// per substruct: 1 = copy to the device, 2 = copy back, both bits possible
static void offload_plan(int layout, int loop, int flags[kMaxSub])
{
    const LayoutDesc &d = kLayouts[layout];
    bool rd[kMaxSub] = {}, out[kMaxSub] = {}, other[kMaxSub] = {};
    for (int f = 0; f < NFIELD; ++f)
        for (int c = 0; c < kNComp[f]; ++c) {
            const int s = d.sub[f][c];
            if (loop_reads(loop, f)) rd[s] = true;
            if (loop_writes(loop, f)) out[s] = true;
            else other[s] = true;
        }
    for (int s = 0; s < d.nsub; ++s) flags[s] = ((rd[s] || (out[s] && other[s])) ? 1 : 0) | (out[s] ? 2 : 0);
}

struct GraphHandle {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

sph_status sph_graph_capture(const sph_plan *p, const sph_store *store, const sph_params *prm,
                             const sph_tuning *tn, void *ws, size_t ws_bytes, void **graph_exec)
{
    if (!graph_exec) return fail(SPH_E_ARG, "graph_exec is null");
    *graph_exec = nullptr;
    hipStream_t cs;
    SPH_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    sph_status s = step_batched(p, store, prm, tn, ws, ws_bytes, cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (s) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t ex;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    *graph_exec = new GraphHandle{g, ex};
    return SPH_OK;
}

sph_status sph_offload_bytes(sph_layout layout, sph_loop loop, int64_t n, size_t *h2d, size_t *d2h)
{
    if ((int)layout < 0 || (int)layout >= kNLayouts) return fail(SPH_E_LAYOUT, "unknown layout");
    sph_status s;
    if ((s = check_loop(loop))) return s;
    if (!h2d || !d2h || n < 0) return fail(SPH_E_ARG, "bad argument");
    int fl[kMaxSub];
    offload_plan(layout, loop, fl);
    size_t a = 0, b = 0;
    for (int k = 0; k < kLayouts[layout].nsub; ++k) {
        const size_t bytes = (size_t)n * kLayouts[layout].sub_bytes[k];
        if (fl[k] & 1) a += bytes;
        if (fl[k] & 2) b += bytes;
    }
    *h2d = a;
    *d2h = b;
    return SPH_OK;
}

sph_status sph_offload_step(const sph_plan *p, const sph_store *host, const sph_store *dev, const sph_params *prm,
                            const sph_tuning *tn, void *ws, size_t ws_bytes, void *stream)
{
    sph_status s;
    if ((s = batched_checks(p, 0)) || (s = check_store(host)) || (s = check_store(dev)) || (s = check_tuning(tn)))
        return s;
    if (!prm) return fail(SPH_E_ARG, "params is null");
    if (host->layout != dev->layout || host->n != p->n || dev->n != p->n)
        return fail(SPH_E_ARG, "host and device stores must share the plan's size and one layout");
    size_t need = 0;
    sph_batched_ws_bytes(p, &need);
    if (!ws || !aligned256(ws)) return fail(SPH_E_ARG, "workspace null or misaligned");
    if (ws_bytes < need) return fail(SPH_E_CAPACITY, "workspace needs " + std::to_string(need) + " bytes");
    if (p->n == 0) return SPH_OK;
    sph_tuning def;
    sph_tuning_default(&def);
    if (!tn) tn = &def;
    hipStream_t st = (hipStream_t)stream;
    char *base = (char *)ws;
    void *q = base;  // queue counter, then the derived planes
    void *pack = base + interact_ws_bytes_for(2, p->n);
    void *res = (char *)pack + pack_bytes_for(2, p->n, p->ntile);
    const LayoutDesc &d = kLayouts[host->layout];
    for (int loop = 0; loop < 3; ++loop) {
        int fl[kMaxSub];
        offload_plan(host->layout, loop, fl);
        for (int k = 0; k < d.nsub; ++k)
            if (fl[k] & 1)
                SPH_HIP(hipMemcpyAsync(dev->sub[k], host->sub[k], (size_t)p->n * d.sub_bytes[k], hipMemcpyHostToDevice, st));
        if ((s = launch_pack(p, loop, dev, true, 0, 0, pack, tn->pack_waves, st, tn->pack_schedule))) return s;
        if ((s = launch_interact(p, loop, true, 0, p->ntask, pack, prm, tn, res, nullptr, q, st))) return s;
        if ((s = launch_unpack(const_cast<sph_plan *>(p), loop, res, true, 0, 0, dev, tn->pack_waves, st,
                               tn->pack_schedule)))
            return s;
        for (int k = 0; k < d.nsub; ++k)
            if (fl[k] & 2)
                SPH_HIP(hipMemcpyAsync(host->sub[k], dev->sub[k], (size_t)p->n * d.sub_bytes[k], hipMemcpyDeviceToHost, st));
    }
    return SPH_OK;
}

// Pipelined offload step.  Three streams: copies to the device, compute, copies
// back.  The particles are cut into nbundle ranges of whole cells; a bundle's
// substructs go to the device on the copy stream, its cells are packed as soon
// as they are there, the interaction waits for every pack, and each bundle is
// unpacked and sent back while the next bundle unpacks and the next loop runs.
// A substruct is sent to the device once per step, before the first loop that
// reads it (or writes part of it); a loop's outputs come back after the loop.
// Every stage runs the same kernels over the same tiles as sph_offload_step.
namespace {
// the events of one call; released when the call returns (an event still
// pending is released by the runtime once it completes)
struct OffloadSync {
    hipStream_t cp = nullptr, dn = nullptr;
    std::vector<hipEvent_t> ev;
    hipEvent_t make()
    {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        ev.push_back(e);
        return e;
    }
    ~OffloadSync()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};
}  // namespace

sph_status sph_offload_step_async(const sph_plan *p, const sph_store *host, const sph_store *dev,
                                  const sph_params *prm, const sph_tuning *tn, int32_t nbundle, void *ws,
                                  size_t ws_bytes, void *stream)
{
    sph_status s;
    if ((s = batched_checks(p, 0)) || (s = check_store(host)) || (s = check_store(dev)) || (s = check_tuning(tn)))
        return s;
    if (!prm) return fail(SPH_E_ARG, "params is null");
    if (host->layout != dev->layout || host->n != p->n || dev->n != p->n)
        return fail(SPH_E_ARG, "host and device stores must share the plan's size and one layout");
    if (nbundle < 1 || nbundle > 64) return fail(SPH_E_ARG, "nbundle outside 1..64");
    size_t need = 0;
    sph_batched_ws_bytes(p, &need);
    if (!ws || !aligned256(ws)) return fail(SPH_E_ARG, "workspace null or misaligned");
    if (ws_bytes < need) return fail(SPH_E_CAPACITY, "workspace needs " + std::to_string(need) + " bytes");
    if (p->n == 0) return SPH_OK;
    sph_tuning def;
    sph_tuning_default(&def);
    if (!tn) tn = &def;
    hipStream_t st = (hipStream_t)stream;
    char *base = (char *)ws;
    void *q = base;
    void *pack = base + interact_ws_bytes_for(2, p->n);
    void *res = (char *)pack + pack_bytes_for(2, p->n, p->ntile);
    const LayoutDesc &d = kLayouts[host->layout];

    // bundles: whole cells, about n / nbundle particles each
    std::vector<int32_t> cb{0};
    for (int b = 1; b < nbundle; ++b) {
        const int64_t target = p->n * b / nbundle;
        int32_t c = cb.back();
        while (c < p->ncell && p->cells[c].first < target) ++c;
        if (c > cb.back() && c < p->ncell) cb.push_back(c);
    }
    cb.push_back(p->ncell);
    const int nb = (int)cb.size() - 1;
    auto part0 = [&](int b) { return b == nb ? p->n : (int64_t)p->cells[cb[b]].first; };

    OffloadSync sy;
    {
        // default-priority streams owned by the plan
        std::lock_guard<std::mutex> lk(const_cast<sph_plan *>(p)->off_mu);
        sph_plan *pm = const_cast<sph_plan *>(p);
        if (!pm->off_h2d) SPH_HIP(hipStreamCreateWithFlags(&pm->off_h2d, hipStreamNonBlocking));
        if (!pm->off_d2h) SPH_HIP(hipStreamCreateWithFlags(&pm->off_d2h, hipStreamNonBlocking));
        sy.cp = pm->off_h2d;
        sy.dn = pm->off_d2h;
    }
    hipEvent_t start = sy.make();
    if (!start) return fail(SPH_E_HIP, "event creation failed");
    SPH_HIP(hipEventRecord(start, st));
    SPH_HIP(hipStreamWaitEvent(sy.cp, start, 0));
    SPH_HIP(hipStreamWaitEvent(sy.dn, start, 0));

    bool on_dev[kMaxSub] = {};
    std::vector<hipEvent_t> back(nb, nullptr);  // last copy-back of each bundle
    for (int loop = 0; loop < 3; ++loop) {
        int fl[kMaxSub];
        offload_plan(host->layout, loop, fl);
        bool send[kMaxSub] = {};
        for (int k = 0; k < d.nsub; ++k) {
            send[k] = (fl[k] & 1) && !on_dev[k];
            if (fl[k] & 1) on_dev[k] = true;
            if (fl[k] & 2) on_dev[k] = true;  // fully written by the unpack
        }
        // 1. bundle copies to the device, each packed once it has arrived
        for (int b = 0; b < nb; ++b) {
            const int64_t p0 = part0(b), p1 = part0(b + 1);
            bool any = false;
            for (int k = 0; k < d.nsub; ++k)
                if (send[k]) {
                    const size_t sb = d.sub_bytes[k];
                    SPH_HIP(hipMemcpyAsync((char *)dev->sub[k] + p0 * sb, (const char *)host->sub[k] + p0 * sb,
                                           (size_t)(p1 - p0) * sb, hipMemcpyHostToDevice, sy.cp));
                    any = true;
                }
            if (any) {
                hipEvent_t e = sy.make();
                if (!e) return fail(SPH_E_HIP, "event creation failed");
                SPH_HIP(hipEventRecord(e, sy.cp));
                SPH_HIP(hipStreamWaitEvent(st, e, 0));
            }
            if ((s = launch_pack_tiles(p, loop, dev, p->tile_off[cb[b]], p->tile_off[cb[b + 1]], pack, tn->pack_waves,
                                       st, tn->pack_schedule)))
                return s;
        }
        // 2. the interaction over every tile
        if ((s = launch_interact(p, loop, true, 0, p->ntask, pack, prm, tn, res, nullptr, q, st))) return s;
        // 3. bundle unpacks, each copied back once unpacked; a bundle is not
        //    unpacked again before its previous copy-back has read it
        for (int b = 0; b < nb; ++b) {
            if (back[b]) SPH_HIP(hipStreamWaitEvent(st, back[b], 0));
            if ((s = launch_unpack_tiles(p, loop, res, p->tile_off[cb[b]], p->tile_off[cb[b + 1]], dev, tn->pack_waves,
                                         st, tn->pack_schedule)))
                return s;
            hipEvent_t u = sy.make();
            hipEvent_t c = sy.make();
            if (!u || !c) return fail(SPH_E_HIP, "event creation failed");
            SPH_HIP(hipEventRecord(u, st));
            SPH_HIP(hipStreamWaitEvent(sy.dn, u, 0));
            const int64_t p0 = part0(b), p1 = part0(b + 1);
            for (int k = 0; k < d.nsub; ++k)
                if (fl[k] & 2) {
                    const size_t sb = d.sub_bytes[k];
                    SPH_HIP(hipMemcpyAsync((char *)host->sub[k] + p0 * sb, (const char *)dev->sub[k] + p0 * sb,
                                           (size_t)(p1 - p0) * sb, hipMemcpyDeviceToHost, sy.dn));
                }
            SPH_HIP(hipEventRecord(c, sy.dn));
            back[b] = c;
        }
    }
    // the caller's stream resumes once both copy streams are done
    hipEvent_t e1 = sy.make(), e2 = sy.make();
    if (!e1 || !e2) return fail(SPH_E_HIP, "event creation failed");
    SPH_HIP(hipEventRecord(e1, sy.cp));
    SPH_HIP(hipEventRecord(e2, sy.dn));
    SPH_HIP(hipStreamWaitEvent(st, e1, 0));
    SPH_HIP(hipStreamWaitEvent(st, e2, 0));
    return SPH_OK;
}

sph_status sph_graph_launch(void *graph_exec, void *stream)
{
    if (!graph_exec) return fail(SPH_E_ARG, "graph_exec is null");
    GraphHandle *h = (GraphHandle *)graph_exec;
    SPH_HIP(hipGraphLaunch(h->exec, (hipStream_t)stream));
    return SPH_OK;
}

void sph_graph_destroy(void *graph_exec)
{
    if (!graph_exec) return;
    GraphHandle *h = (GraphHandle *)graph_exec;
    (void)hipGraphExecDestroy(h->exec);
    (void)hipGraphDestroy(h->graph);
    delete h;
}

}  // extern "C"
