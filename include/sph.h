/*
 * sph.h -- C-ABI of libsph, the MI355X (gfx950) pack / interact / unpack path
 * for smoothed particle hydrodynamics.
 *
 * The paper this follows ("Memory Layouts for GPU-Data Transfer Buffering in
 * SPH") offloads SPH interaction loops in bundles of cell tasks: each task's
 * particle attributes are *packed* into a compact buffer, the interactions are
 * computed on the GPU (the *launch*), and the results are *unpacked* with
 * reductions back into the particles (Sec. 2.3).  Three loops run per step --
 * density, gradient and force -- each reading and writing its own attribute
 * set (Sec. 2.1, Table 1).  The particle store may be laid out as AoS, a
 * randomly ordered AoS, split AoS grouped by access pattern (pack-gradient,
 * pack-force, pack-shared), the same split again by data type, or SoA
 * (Sec. 3.1), hidden behind getters and setters (Sec. 3.2, Algorithm 1).
 *
 * Conventions shared by every call
 *  - Every call returns sph_status; nothing throws across the ABI.  On an
 *    error nothing has been enqueued and no memory has been written, except
 *    where a call says otherwise (sph_step_kdk stopping for a plan rebuild
 *    after its drift; a HIP failure in the middle of a multi-launch call).
 *  - Device pointers are HIP device (or host-mapped) addresses owned by the
 *    caller; the library never frees caller memory.  Store substruct arrays
 *    and buffers must be 256-byte aligned.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    asynchronously on it; faults inside kernels surface at the caller's next
 *    synchronisation.  Calls that return a device-side result to the host
 *    (sph_drift with its outputs, sph_cfl_dt, sph_h_iterate, sph_step_kdk)
 *    synchronise the stream.  HIP errors map to SPH_E_HIP, detail in
 *    sph_last_error().
 *  - Plans are library-owned and immutable after creation; one plan may be used
 *    from several threads and streams at once.  No call keeps global mutable
 *    state besides the thread-local error text and, for
 *    sph_step_batched_noalloc, one static device scratch array per GPU.
 *  - Floating point: pack and unpack are bit-exact data movement (one FP64
 *    subtraction rounded once to FP32 for positions; FP32 additions in a fixed
 *    order for reductions).  Interaction sums are FP32.
 */
#ifndef SPH_H
#define SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sph_status {
    SPH_OK = 0,
    SPH_E_ARG = -1,         /* null / misaligned pointer, bad enum, bad range        */
    SPH_E_LAYOUT = -2,      /* unknown layout, or a store that does not match the   */
                            /* layout's substruct count                            */
    SPH_E_CAPACITY = -3,    /* a caller buffer is smaller than the call needs        */
    SPH_E_PLAN = -4,        /* cells / tasks inconsistent (index out of range, ...)  */
    SPH_E_HIP = -5,         /* a HIP runtime call failed                             */
    SPH_E_UNSUPPORTED = -6  /* valid request the plan cannot serve                   */
} sph_status;

/* Particle layouts (Sec. 3.1).  The substructs of each, member order and byte
 * offsets are fixed by the library and reported by sph_layout_info() and
 * sph_field_location(); see those calls for the exact tables. */
typedef enum sph_layout {
    SPH_AOS = 0,              /* one 160-byte record, members in usage order      */
    SPH_AOS_RANDOM = 1,       /* the same members in a fixed shuffled order        */
    SPH_SAOS_GRAD = 2,        /* gradient-pack set in one substruct                */
    SPH_SAOS_FORCE = 3,       /* force-pack set in one substruct                   */
    SPH_SAOS_SHARED = 4,      /* {x, m, h} shared by all loops in its own substruct */
    SPH_SAOS_GRAD_TYPE = 5,   /* SAOS_GRAD split again by data type                */
    SPH_SAOS_FORCE_TYPE = 6,  /* SAOS_FORCE split again by data type               */
    SPH_SAOS_SHARED_TYPE = 7, /* SAOS_SHARED split again by data type              */
    SPH_SOA = 8,              /* one array per scalar component                    */
    SPH_SAOS_SHARED_REPL = 9, /* SAOS_SHARED with the position replicated into   */
                              /* every substruct a loop packs from (Sec. 5's data */
                              /* replication): {x m h} {x v u rho} {x rho_dh D R  */
                              /* alpha_v alpha_d} {outputs} {cold}                */
    SPH_NLAYOUTS = 10
} sph_layout;

typedef enum sph_loop { SPH_DENSITY = 0, SPH_GRADIENT = 1, SPH_FORCE = 2 } sph_loop;

/* Logical particle fields (Table 1 plus the outputs the loops produce).
 * Component type: X float64[3]; V, A, ROT float32[3]; TIME_BIN int8;
 * ID int64; COLD 40 opaque bytes (5 x uint64) no loop touches; the rest float32. */
typedef enum sph_field {
    SPH_F_X = 0, SPH_F_V, SPH_F_A, SPH_F_MASS, SPH_F_H, SPH_F_U, SPH_F_U_DT, SPH_F_RHO,
    SPH_F_RHO_DH, SPH_F_WCOUNT, SPH_F_DIV, SPH_F_ROT, SPH_F_LAP, SPH_F_VSIG, SPH_F_ALPHA_V,
    SPH_F_ALPHA_D, SPH_F_TIME_BIN, SPH_F_ID, SPH_F_COLD, SPH_NFIELDS
} sph_field;

#define SPH_MAX_SUB 32

/* A particle store: `nsub` caller-owned substruct arrays, each holding n
 * records of sph_layout_info()'s sub_bytes[s] bytes.  256-byte aligned. */
typedef struct sph_store {
    int32_t layout;
    int32_t nsub;
    int64_t n;
    void *sub[SPH_MAX_SUB];
} sph_store;

/* A cell (octree leaf or grid cell, Sec. 2.2): particles [first, first+count)
 * of the store, all inside the cube [loc, loc + width). 48 bytes. */
typedef struct sph_cell {
    double loc[3];
    double width;
    int64_t first;
    int32_t count;
    int32_t pad;
} sph_cell;

/* A task (Sec. 2.2): a self task (ci == cj, shift = 0) or a pair task whose
 * cj particles are used at x + shift (the periodic image next to ci). 40 bytes. */
typedef struct sph_task {
    int32_t ci, cj;
    int32_t pad[2];
    double shift[3];
} sph_task;

/* Physics constants (defaults 5/3, 3, 1e-4). */
typedef struct sph_params {
    float gamma_ad;
    float beta_visc;
    float balsara_eps;
    float pad;
} sph_params;

/* Launch parameters of the batched form (sph_tuning_default fills them). */
typedef struct sph_tuning {
    int32_t blocks_per_cu;   /* persistent grid = 4 x blocks_per_cu x CU count waves
                                of the interaction kernels (1..64)                 */
    int32_t window[3];       /* candidate window per wave for density, gradient and
                                force: 128, 256 or 512 candidates (512: not force) */
    int32_t pack_waves;      /* waves per block in pack / unpack kernels (1..8)     */
    int32_t queue;           /* 0 = static stride; 1 = one device work queue in
                                descending cost order; 2 = one queue per XCD over
                                a spatially contiguous share of the tiles (equal
                                estimated cost each), stealing from the other
                                shares once its own is drained                     */
    int32_t blocks_per_loop[3]; /* per loop (density, gradient, force): 1..64 replaces
                                blocks_per_cu for that loop's kernel, 0 keeps it    */
    int32_t pack_schedule;   /* loop fission of the batched pack and unpack (Sec.
                                3.3): 0 by particle (one kernel converts every
                                field), 1 by struct (one kernel per substruct), 2
                                by element (one per field), 3 by type (one per
                                component type), 4 by struct and type; the groups
                                of a layout and loop are sph_fission_passes()'s   */
} sph_tuning;

typedef struct sph_plan sph_plan; /* library-owned, opaque */

/* Plan statistics. */
typedef struct sph_plan_info {
    int64_t n;            /* particles                                         */
    int32_t ncell, ntask;
    int64_t nslot;        /* slots over all tasks (a particle per task side)    */
    int64_t nchunk;       /* 64-slot chunks over all tasks                      */
    int32_t ntile;        /* 64-particle tiles over all cells                   */
    int32_t max_cell;     /* largest cell                                        */
    int32_t max_nbr;      /* most neighbour cells of one cell (incl. itself)     */
    int32_t batched_ok;   /* cells tile the store in order (batched form usable) */
    int32_t mixed_widths; /* cells of more than one width: the force loop then  */
                          /* tests mixed supports with two matrix-core products */
    int32_t pad;
} sph_plan_info;

/* ---------------------------------------------------------------------- */
/* Error text and layout queries (host only, no GPU needed).               */
/* ---------------------------------------------------------------------- */
const char *sph_status_str(sph_status s);
/* Detail of the last failure on the calling thread ("" if none). */
const char *sph_last_error(void);

/* Substruct count and record bytes of a layout (Sec. 3.1).  sub_bytes must
 * hold SPH_MAX_SUB entries.  Members sit at natural alignment in the listed
 * order, each record padded to 8 bytes (SoA: one array per scalar component,
 * element size = component size). */
sph_status sph_layout_info(sph_layout layout, int32_t *nsub, size_t *sub_bytes);

/* Where component `comp` of `field` lives: substruct index, byte offset in the
 * record and record stride (the getter/setter mapping of Algorithm 1).  For
 * a layout that replicates x this is the primary copy (the first in member
 * order), which every read takes; every write of x (sph_store_put, the
 * drift, sph_store_convert) writes all copies, and sph_x_replicas lists the
 * others. */
/* Copies of x beyond the primary one: *count of them, replica r in substruct
 * sub[r] at byte offset offset[r] of the record (component c 8 bytes further);
 * sub and offset hold at least 3 entries. */
sph_status sph_x_replicas(sph_layout layout, int32_t *count, int32_t *sub, size_t *offset);
sph_status sph_field_location(sph_layout layout, sph_field field, int32_t comp, int32_t *sub,
                              size_t *offset, size_t *stride);

/* Components and bytes per component of a field. */
sph_status sph_field_info(sph_field field, int32_t *ncomp, int32_t *comp_bytes);

/* Packed record of a loop (Table 1): planes of float32, plane k holding
 * plane_floats[k] floats per slot.  A buffer for P slots stores plane k at
 * byte offset P * 4 * (sum of plane_floats before k), slot s of plane k at
 * s * 4 * plane_floats[k] inside it:
 *   density : [dx dy dz h] [m]
 *   gradient: [dx dy dz h] [vx vy vz m] [u rho]
 *   force   : [dx dy dz h] [vx vy vz m] [u rho rho_dh D] [R0 R1 R2 alpha_v] [alpha_d]
 * (dx,dy,dz) = float32(x - o) computed in float64 and rounded once to nearest,
 * o = loc(ci) for ci's particles and loc(ci) - shift for cj's (the periodic
 * pre-processing of Sec. 2.3).  Results are float planes per slot:
 *   density [rho rho_dh wcount]; gradient [D R0 R1 R2 L V]; force [a0 a1 a2 u_dt]. */
sph_status sph_pack_layout(sph_loop loop, int32_t *nplane, int32_t *plane_floats, int32_t *result_planes);

/* Loop fission (Sec. 3.3): the kernels one pack and one unpack of the
 * batched form run under sph_tuning.pack_schedule (0..4, as listed there),
 * each given by the members it converts.  A pack mask has bit k set for the
 * k-th float of the force record (dx dy dz h vx vy vz m u rho rho_dh D R0 R1
 * R2 alpha_v alpha_d); density and gradient pack subsets of it.  An unpack
 * mask has bit k set for result plane k of the loop.  Each loop's members are
 * split into groups that share what the schedule keys on (nothing, the
 * substruct, the field, the component's type, substruct and type), the groups
 * in the order of their first member; the masks partition the loop's members.
 * pack_masks and unpack_masks hold SPH_MAX_PASSES entries.  Host only. */
#define SPH_MAX_PASSES 32
sph_status sph_fission_passes(sph_layout layout, sph_loop loop, int32_t schedule, int32_t *npack,
                              uint32_t *pack_masks, int32_t *nunpack, uint32_t *unpack_masks);

/* ---------------------------------------------------------------------- */
/* Store access: the getter / setter analogue (Sec. 3.2, Algorithm 1).      */
/* ---------------------------------------------------------------------- */
/* Copy a dense device array src[n][ncomp] of the field's type into the store. */
sph_status sph_store_put(const sph_store *store, sph_field field, const void *src, void *stream);
/* Copy a field out of the store into a dense device array dst[n][ncomp]. */
sph_status sph_store_get(const sph_store *store, sph_field field, void *dst, void *stream);
/* Rewrite a store into another layout (a decomposition that changes with the
 * algorithmic phase, Sec. 4's Recommendation 3): every component of every
 * field of every particle is copied bit for bit from src into dst, the
 * padding bytes of dst's records are set to zero.  Both are device stores of
 * the same n, in any two layouts (the same one included); no substruct of dst
 * may overlap one of src (SPH_E_ARG).  One kernel, one thread per particle:
 * each source record read once, each destination record written once. */
sph_status sph_store_convert(const sph_store *src, const sph_store *dst, void *stream);

/* ---------------------------------------------------------------------- */
/* Plan: cells and tasks of one step (Sec. 2.2).                            */
/* ---------------------------------------------------------------------- */
/* Validate host arrays cells[ncell], tasks[ntask] over n particles and upload
 * them with derived tables to the current device.  Every task's cells must be
 * in range, self tasks must carry a zero shift, cells must lie inside [0, n).
 * Errors: SPH_E_ARG (null / negative sizes), SPH_E_PLAN, SPH_E_HIP. */
sph_status sph_plan_create(const sph_cell *cells, int32_t ncell, const sph_task *tasks,
                           int32_t ntask, int64_t n, sph_plan **out);
void sph_plan_destroy(sph_plan *plan);
sph_status sph_plan_get_info(const sph_plan *plan, sph_plan_info *info);
/* Reach of every cell (reach: host array of ncell doubles): the smallest gap,
 * minimum image in the unit box, between the cell's cube and the cube of a
 * non-empty cell it shares no task with, at most 1/2 (and at most 1/G where
 * the plan buckets cells on a G^3 grid no finer than the widest cell).  Any
 * particle of the cell, while inside its cube, finds every neighbour within
 * this distance through the cell's tasks (Sec. 2.2): the smoothing-length
 * step holds each support to it, and the kick-drift-kick step checks that
 * supports plus drift stay within it.  On a uniform grid with self and 26
 * neighbour tasks it is the cell width. */
sph_status sph_plan_cell_reach(const sph_plan *plan, double *reach);
/* Slots of tasks [t0, t1) and the bytes a pack / result buffer for that range
 * needs (planes hold P = nslot rounded up to 64 slots; the pack buffer also
 * carries 32 bytes of tile bounds per 64-slot chunk after the planes). */
sph_status sph_plan_buffer_bytes(const sph_plan *plan, sph_loop loop, int32_t t0, int32_t t1,
                                 int64_t *nslot, size_t *pack_bytes, size_t *result_bytes);

/* ---------------------------------------------------------------------- */
/* Per-task / bundled path: any task range [t0, t1) is one bundle.          */
/* ---------------------------------------------------------------------- */
/* Set the loop's outputs in the store to +0.0f (before the first unpack). */
sph_status sph_zero_outputs(const sph_plan *plan, sph_loop loop, const sph_store *store, void *stream);

/* Pack the slots of tasks [t0, t1) in task order -- ci's particles, then cj's,
 * each in store order -- into pack_buf (pack_bytes from sph_plan_buffer_bytes). */
sph_status sph_pack(const sph_plan *plan, sph_loop loop, const sph_store *store, int32_t t0,
                    int32_t t1, void *pack_buf, size_t pack_bytes, void *stream);

/* Interaction loops over a packed range (Sec. 2.1).  For every slot i of a
 * task, sum over the slots j of the other cell of the task (the same cell for
 * a self task) and write the slot's partial results to res_buf:
 *   density : j with r < H_i, i itself included
 *   gradient: j != i with r < H_i
 *   force   : j != i with r < max(H_i, H_j)
 * H = sqrt(10/3) h.  counts (optional, int32 per slot) receives the number of
 * interacting j; a non-null counts selects kernels that apply the exact
 * support and j != i tests before every pair term, while without counts the
 * kernels skip tests whose pairs contribute exact zeros anyway (the sums agree
 * to rounding).  pack_bytes / res_bytes are the caller's buffer sizes. */
sph_status sph_density(const sph_plan *plan, const void *pack_buf, size_t pack_bytes, int32_t t0,
                       int32_t t1, const sph_params *params, void *res_buf, size_t res_bytes,
                       int32_t *counts, void *stream);
sph_status sph_gradient(const sph_plan *plan, const void *pack_buf, size_t pack_bytes, int32_t t0,
                        int32_t t1, const sph_params *params, void *res_buf, size_t res_bytes,
                        int32_t *counts, void *stream);
sph_status sph_force(const sph_plan *plan, const void *pack_buf, size_t pack_bytes, int32_t t0,
                     int32_t t1, const sph_params *params, void *res_buf, size_t res_bytes,
                     int32_t *counts, void *stream);

/* Reduce the partial results of tasks [t0, t1) into the store in ascending
 * task order (ci's slots, then cj's): FP32 additions, and the larger value for
 * the signal velocity V (Sec. 2.3, unpacking with reductions). */
sph_status sph_unpack(const sph_plan *plan, sph_loop loop, const void *res_buf, size_t res_bytes,
                      int32_t t0, int32_t t1, const sph_store *store, void *stream);

/* Per-task driver: for every task t in [t0, t1), in order, one pack, one
 * interaction and one unpack launch over [t, t+1) -- the paper's offload
 * cycle with one task per bundle -- after zeroing the loop's outputs when
 * zero_first is set.  pack_buf / res_buf must hold the largest single task. */
sph_status sph_run_per_task(const sph_plan *plan, sph_loop loop, const sph_store *store, int32_t t0,
                            int32_t t1, int32_t zero_first, const sph_params *params, void *pack_buf,
                            size_t pack_bytes, void *res_buf, size_t res_bytes, void *stream);
/* Bytes of the pack and result buffers of the largest single task. */
sph_status sph_plan_task_max_bytes(const sph_plan *plan, sph_loop loop, size_t *pack_bytes,
                                   size_t *result_bytes);

/* ---------------------------------------------------------------------- */
/* Batched form: all tasks of a step per launch (the paper's bundling of    */
/* ready tasks, Sec. 2.3, taken to one bundle per step).  Each cell is      */
/* packed once (slot = particle index, origin = the cell's own loc), every  */
/* particle gathers over all its neighbour cells in one work item pulled    */
/* from a device queue, and unpack writes each result once.  Requires cells */
/* that tile the store in order (sph_plan_info.batched_ok).                 */
/* ---------------------------------------------------------------------- */
void sph_tuning_default(sph_tuning *t);
/* Workspace for sph_step_batched / sph_graph_capture. */
sph_status sph_batched_ws_bytes(const sph_plan *plan, size_t *bytes);
/* Individual stages (buffers as for the per-task path with P = n rounded up). */
sph_status sph_pack_cells(const sph_plan *plan, sph_loop loop, const sph_store *store, void *pack_buf,
                          size_t pack_bytes, const sph_tuning *tuning, void *stream);
/* Workspace of sph_interact_cells for a loop: 256 bytes for the work-queue
 * counters (one per XCD), then (gradient, force) per-particle planes of the
 * quantities the pair terms derive from the packed fields, computed once per
 * particle by the same launch: gradient u, m/rho and the sound speed; force
 * 1/H, the spline normalisation H^-5 8/pi, A = P/(Omega rho^2), the sound
 * speed, the Balsara-limited viscosity switch, alpha_d, rho and u (with the
 * pair term's constant factors folded in). */
sph_status sph_interact_ws_bytes(const sph_plan *plan, sph_loop loop, size_t *bytes);
/* ws: device memory of ws_bytes >= sph_interact_ws_bytes(loop), 256-byte
 * aligned, owned by the caller; overwritten. */
sph_status sph_interact_cells(const sph_plan *plan, sph_loop loop, const void *pack_buf,
                              size_t pack_bytes, const sph_params *params, const sph_tuning *tuning,
                              void *res_buf, size_t res_bytes, int32_t *counts, void *ws,
                              size_t ws_bytes, void *stream);
/* out = +0.0f + result (V: the larger of +0.0f and the result). */
sph_status sph_unpack_cells(const sph_plan *plan, sph_loop loop, const void *res_buf, size_t res_bytes,
                            const sph_store *store, const sph_tuning *tuning, void *stream);
/* density -> gradient -> force over the whole store, in stages: pack the
 * density record, density, pack the gradient record (rho taken from the
 * density results), gradient, pack the force record (rho, rho_dh, D, R from
 * the earlier results, the force pair term's derived per-particle planes
 * written beside it), force, then one write-back of every output into the
 * store -- the unpacks of Sec. 2.3 folded into one pass at the end of the
 * step.  The store ends bit for bit as after pack -> interact -> unpack per
 * loop (sph_pack_cells / sph_interact_cells / sph_unpack_cells).  With a
 * loop-fission pack schedule (tuning->pack_schedule != 0) every loop is
 * unpacked into the store before the next packs from it.  ws: device memory
 * of sph_batched_ws_bytes, 256-byte aligned, caller-owned, overwritten. */
sph_status sph_step_batched(const sph_plan *plan, const sph_store *store, const sph_params *params,
                            const sph_tuning *tuning, void *ws, size_t ws_bytes, void *stream);
/* The stages of sph_step_batched, one call each (same ws; the step's result
 * planes and pack buffer live in it): sph_step_pack for density, gradient,
 * force in turn, each followed by sph_step_interact of the same loop, then
 * sph_step_writeback.  Results between the calls live in ws; a gradient or
 * force pack that loads a substruct record whole and finds outputs of earlier
 * loops in it writes the record back with them (SAOS_SHARED: rho with
 * {v u rho}, rho_dh, D, R with the force-only substruct; SoA: their arrays),
 * and the write-back stores the rest, so the store is complete only after
 * sph_step_writeback. */
sph_status sph_step_pack(const sph_plan *plan, sph_loop loop, const sph_store *store,
                         const sph_params *params, const sph_tuning *tuning, void *ws, size_t ws_bytes,
                         void *stream);
sph_status sph_step_interact(const sph_plan *plan, sph_loop loop, const sph_params *params,
                             const sph_tuning *tuning, void *ws, size_t ws_bytes, void *stream);
sph_status sph_step_writeback(const sph_plan *plan, const sph_store *store, const sph_tuning *tuning,
                              void *ws, size_t ws_bytes, void *stream);
/* Which stage of the staged step stores each output into a store of this
 * layout: writer[13] in the order rho, rho_dh, wcount, D, R[3], lap_u, v_sig,
 * a[3], u_dt; 1 or 2 = the gradient or force pack, 3 = the write-back. */
sph_status sph_step_output_writers(sph_layout layout, int32_t *writer);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the step of
 * sph_step_batched with its workspace taken from a static per-device scratch
 * array of SPH_NOALLOC_SCRATCH_BYTES inside the library (one copy per GPU the
 * library runs on, held until the process ends), so the call allocates
 * nothing.  The caller still provides the plan and the store.  A plan whose
 * sph_batched_ws_bytes exceeds the scratch size is refused with
 * SPH_E_CAPACITY before anything is enqueued.  Every call on one GPU shares
 * that GPU's scratch: calls that overlap on one GPU (other streams, other
 * threads, graph replays in flight) race and must be ordered by the caller.
 * The first call on a device looks up that device's scratch address (the
 * device must be current). */
#define SPH_NOALLOC_SCRATCH_BYTES (64u << 20)
sph_status sph_step_batched_noalloc(const sph_plan *plan, const sph_store *store, const sph_params *params,
                                    const sph_tuning *tuning, void *stream);
/* Smoothing-length iteration: the per-particle update between the density
 * and gradient loops (Sec. 2.1's linear kernels) that makes every h
 * consistent with its density, rho(h) h^3 = m eta^3 (h = eta (m/rho)^(1/3);
 * eta = 1.2348 gives about 48 neighbours for the cubic spline).  Each pass
 * runs the density loop (batched form; after the first pass only over the
 * tiles holding a particle that moved), then one Newton step per particle on
 * f(h) = rho h^3 - m eta^3 using the density and its h-derivative rho_dh: a
 * particle whose step is at most tol h keeps its h and the density computed
 * with it; any other moves to h + dh, limited to [h/2, 2h]; every h is then
 * held to a support gamma_K h no wider than its own cell.  Stops when no particle moved or after
 * max_iter passes; *iterations receives the passes run and *unconverged the
 * particles that still moved in the last one (their density belongs to their
 * previous h).  The store's h, rho, rho_dh and wcount are updated in place.
 * Synchronises `stream` once per pass (the host reads the count); not
 * capturable.  ws: device memory of sph_h_iterate_ws_bytes bytes, 256-byte
 * aligned, owned by the caller.  iterations / unconverged may be null. */
sph_status sph_h_iterate_ws_bytes(const sph_plan *plan, size_t *bytes);
sph_status sph_h_iterate(const sph_plan *plan, const sph_store *store, const sph_params *params,
                         const sph_tuning *tuning, float eta, float tol, int32_t max_iter, void *ws,
                         size_t ws_bytes, int32_t *iterations, int64_t *unconverged, void *stream);
/* Time integration around the loops (the step the loops serve, Sec. 2.1):
 * a kick-drift-kick leapfrog with one global time step.  Operations are
 * exactly as written, each rounded once, no fused multiply-add.
 * sph_kick: v += a dt and u += u_dt dt in float32 (a, u_dt from the last
 * force loop).  sph_drift: x += v dt in float64 (v widened exactly); with
 * max_outside / max_h non-null it also returns, after synchronising `stream`,
 * the largest distance (float64) by which a particle now lies outside its
 * cell's cube and the largest h.  sph_cfl_dt: dt = min over particles with
 * V > 0 of (cfl (gamma_K h)) / V, float32 (V the signal velocity of the last
 * gradient loop; +inf if none), synchronises `stream`.  sph_step_kdk: kick by
 * dt/2 and drift by dt (one pass over the particles), then -- if gamma_K max h + 2 max_outside does not exceed
 * the narrowest cell, so every pair within a support still meets in adjacent
 * cells -- density, gradient and force (sph_step_batched) and a second kick by
 * dt/2; otherwise it stops after the drift with *rebuild = 1 and SPH_E_PLAN:
 * the caller rebuilds the plan from the drifted positions, runs the loops and
 * the second kick.  Synchronises `stream` once (the reach check).  ws:
 * sph_integrate_ws_bytes bytes for sph_drift / sph_cfl_dt; for sph_step_kdk
 * sph_batched_ws_bytes rounded up to 256, then sph_integrate_ws_bytes. */
sph_status sph_integrate_ws_bytes(const sph_plan *plan, size_t *bytes);
sph_status sph_kick(const sph_store *store, float dt, void *stream);
sph_status sph_drift(const sph_plan *plan, const sph_store *store, double dt, void *ws, size_t ws_bytes,
                     double *max_outside, float *max_h, void *stream);
sph_status sph_cfl_dt(const sph_plan *plan, const sph_store *store, float cfl, void *ws, size_t ws_bytes,
                      float *dt, void *stream);
sph_status sph_step_kdk(const sph_plan *plan, const sph_store *store, const sph_params *params,
                        const sph_tuning *tuning, float dt, void *ws, size_t ws_bytes, int32_t *rebuild,
                        void *stream);
/* Capture sph_step_batched into an executable HIP graph (*graph_exec). */
sph_status sph_graph_capture(const sph_plan *plan, const sph_store *store, const sph_params *params,
                             const sph_tuning *tuning, void *ws, size_t ws_bytes, void **graph_exec);
sph_status sph_graph_launch(void *graph_exec, void *stream);
void sph_graph_destroy(void *graph_exec);

/* ---------------------------------------------------------------------- */
/* Offload form (Sec. 2.3's launch: H2D, compute, D2H).  `host` is the      */
/* authoritative store in pinned host memory, `dev` a device store of the   */
/* same layout.  For each loop: copy host -> device every substruct holding  */
/* a field the loop's pack reads, or holding one of its outputs together    */
/* with other fields; run pack -> interaction -> unpack (batched form); copy */
/* device -> host every substruct holding one of the loop's outputs.  All    */
/* copies are stream-ordered hipMemcpyAsync.                                 */
/* ---------------------------------------------------------------------- */
/* Bytes moved each way for one loop over n particles of a layout. */
sph_status sph_offload_bytes(sph_layout layout, sph_loop loop, int64_t n, size_t *h2d_bytes,
                             size_t *d2h_bytes);
/* One offload step (density, gradient, force).  ws as for sph_step_batched. */
sph_status sph_offload_step(const sph_plan *plan, const sph_store *host, const sph_store *dev,
                            const sph_params *params, const sph_tuning *tuning, void *ws, size_t ws_bytes,
                            void *stream);
/* The same step pipelined (Sec. 2.3's cycle with its transfers overlapped):
 * the particles are cut into nbundle (1..64) ranges of whole cells; on a copy
 * stream each substruct a step needs goes to the device once, bundle by bundle,
 * before the first loop that reads (or partly writes) it; each bundle is packed
 * as soon as its bytes are there; the interaction waits for every pack; each
 * bundle is then unpacked and its output substructs copied back on a second
 * copy stream while the rest of the work proceeds.  The copy streams belong to
 * the plan (created on the first call, default priority, destroyed with the
 * plan); the call is ordered after earlier work on `stream`, and later work on
 * `stream` is ordered after all of it.  The host store must not change during
 * the call; on completion host and device stores hold what sph_offload_step
 * leaves (every kernel runs over the same tiles).  Calls sharing a plan must not
 * overlap.  ws as for sph_step_batched. */
sph_status sph_offload_step_async(const sph_plan *plan, const sph_store *host, const sph_store *dev,
                                  const sph_params *params, const sph_tuning *tuning, int32_t nbundle,
                                  void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------- */
/* Adjoint of L = sum_i |a_i|^2 through density and force (hand-written),   */
/* the differentiable form of the loops of Sec. 2.1.                        */
/* The artificial-viscosity switch alpha~ = alpha_v B and alpha_d are held  */
/* fixed; h and u are constants.  Inputs are per-particle device arrays in  */
/* store order: x float64[n][3], v float32[n][3], m, h, u, atilde, alpha_d  */
/* float32[n].  Arithmetic is float64, since a and the small components   */
/* of the gradient are sums of nearly cancelling pair terms, and the        */
/* outputs are float64.  The plan's cells must tile the store in order; */
/* ws (sph_adjoint_ws_bytes, 256-byte aligned) is scratch overwritten by    */
/* every call.  All calls are asynchronous on `stream`.                     */
/* ---------------------------------------------------------------------- */
/* Forward: rho, rho_dh (float64[n]), a (float64[n][3]), u_dt (float64[n]). */
sph_status sph_adjoint_forward(const sph_plan *plan, const double *x, const float *v, const float *m,
                               const float *h, const float *u, const float *atilde,
                               const float *alpha_d, const sph_params *params, double *rho,
                               double *rho_dh, double *a, double *u_dt, void *ws, size_t ws_bytes,
                               void *stream);
/* Backward of force: given a_bar = dL/da (float64[n][3]), recomputes the
 * density of x (pair terms and densities are never stored between calls) and
 * writes (overwrites) the force loop's contributions to dL/dx (float64[n][3]),
 * dL/dv (float64[n][3]) and dL/dm (float64[n]), and rho_bar = dL/drho,
 * rhodh_bar = dL/drho_dh (float64[n]). */
sph_status sph_force_adjoint(const sph_plan *plan, const double *x, const float *v, const float *m,
                             const float *h, const float *u, const float *atilde,
                             const float *alpha_d, const sph_params *params, const double *a_bar,
                             double *x_bar, double *v_bar, double *m_bar, double *rho_bar,
                             double *rhodh_bar, void *ws, size_t ws_bytes, void *stream);
/* Backward of density: accumulates (+=) dL/dx and dL/dm (float64) from
 * rho_bar, rhodh_bar. */
sph_status sph_density_adjoint(const sph_plan *plan, const double *x, const float *m, const float *h,
                               const double *rho_bar, const double *rhodh_bar, double *x_bar,
                               double *m_bar, void *ws, size_t ws_bytes, void *stream);
/* Workspace of the three adjoint calls. */
sph_status sph_adjoint_ws_bytes(const sph_plan *plan, size_t *bytes);

#ifdef __cplusplus
}
#endif
#endif /* SPH_H */
