/*
 * sph_abi_client.c -- a plain C99 client of libsph that uses nothing but
 * include/sph.h and the HIP runtime's memory calls.
 *
 *   sph_abi_client tables
 *       Prints, one line each, the status strings, every layout's substruct
 *       sizes, every field's location in every layout, the packed record of
 *       each loop and the default launch parameters, then the status of calls
 *       with invalid arguments (they must fail before touching a device).
 *   sph_abi_client step IN OUT
 *       Reads a particle set with its cells and tasks from IN, puts it into a
 *       device store of the requested layout, runs one batched
 *       density -> gradient -> force step (sph_step_batched, default launch
 *       parameters and physics constants) and writes every output field to
 *       OUT.
 *   sph_abi_client per_task IN OUT BUNDLE
 *       The same through the per-task calls: for each loop in turn,
 *       sph_zero_outputs, then for every bundle of BUNDLE consecutive tasks
 *       sph_pack -> sph_density / sph_gradient / sph_force -> sph_unpack.
 *
 * IN (little endian): int64 n, int32 ncell, int32 ntask, int32 layout,
 * int32 0; ncell sph_cell records; ntask sph_task records; then x (n x 3
 * float64), v (n x 3 float32), mass, h, u, alpha_v, alpha_d (n float32 each).
 * OUT: rho, rho_dh, wcount, div_v, rot_v (n x 3), lap_u, v_sig, a (n x 3),
 * u_dt, each float32.  Exit status 0 on success, 1 on any failure (with the
 * failing call and the library's error text on stderr).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "sph.h"

#define CHECK(call)                                                                              \
    do {                                                                                         \
        sph_status s_ = (call);                                                                  \
        if (s_ != SPH_OK) {                                                                      \
            fprintf(stderr, "%s: %s (%s)\n", #call, sph_status_str(s_), sph_last_error());       \
            exit(1);                                                                             \
        }                                                                                        \
    } while (0)

#define HIPCHECK(call)                                                                           \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));                           \
            exit(1);                                                                             \
        }                                                                                        \
    } while (0)

static void read_all(FILE *f, void *dst, size_t bytes)
{
    if (bytes && fread(dst, 1, bytes, f) != bytes) {
        fprintf(stderr, "short input file\n");
        exit(1);
    }
}

static void *host_alloc(size_t bytes)
{
    void *p = malloc(bytes ? bytes : 1);
    if (!p) {
        fprintf(stderr, "out of host memory\n");
        exit(1);
    }
    return p;
}

static int tables(void)
{
    int32_t i, f, c, l;
    for (i = 0; i >= -6; --i) printf("status %d %s\n", i, sph_status_str((sph_status)i));
    for (l = 0; l < SPH_NLAYOUTS; ++l) {
        int32_t nsub = 0;
        size_t bytes[SPH_MAX_SUB];
        CHECK(sph_layout_info((sph_layout)l, &nsub, bytes));
        printf("layout %d %d", l, nsub);
        for (i = 0; i < nsub; ++i) printf(" %zu", bytes[i]);
        printf("\n");
        for (f = 0; f < SPH_NFIELDS; ++f) {
            int32_t ncomp = 0, cb = 0;
            CHECK(sph_field_info((sph_field)f, &ncomp, &cb));
            for (c = 0; c < ncomp; ++c) {
                int32_t sub = -1;
                size_t off = 0, stride = 0;
                CHECK(sph_field_location((sph_layout)l, (sph_field)f, c, &sub, &off, &stride));
                printf("field %d %d %d %d %zu %zu\n", l, f, c, sub, off, stride);
            }
        }
    }
    for (l = 0; l < 3; ++l) {
        int32_t np = 0, pf[32], rp = 0;
        CHECK(sph_pack_layout((sph_loop)l, &np, pf, &rp));
        printf("pack %d %d", l, rp);
        for (i = 0; i < np; ++i) printf(" %d", pf[i]);
        printf("\n");
    }
    {
        sph_tuning t;
        sph_tuning_default(&t);
        printf("tuning %d %d %d %d %d %d %d %d %d %d\n", t.blocks_per_cu, t.window[0], t.window[1], t.window[2],
               t.pack_waves, t.queue, t.blocks_per_loop[0], t.blocks_per_loop[1], t.blocks_per_loop[2],
               t.pack_schedule);
    }
    {
        /* invalid arguments: rejected on the host */
        sph_plan *plan = NULL;
        sph_cell cell;
        sph_task task;
        int32_t nsub = 0;
        size_t bytes[SPH_MAX_SUB];
        memset(&cell, 0, sizeof cell);
        memset(&task, 0, sizeof task);
        printf("invalid plan_null_cells %d\n", (int)sph_plan_create(NULL, 1, &task, 1, 1, &plan));
        printf("invalid plan_negative_n %d\n", (int)sph_plan_create(&cell, 1, &task, 1, -1, &plan));
        cell.count = 4;
        task.ci = 0;
        task.cj = 3;
        printf("invalid plan_task_cell %d\n", (int)sph_plan_create(&cell, 1, &task, 1, 4, &plan));
        printf("invalid layout %d\n", (int)sph_layout_info((sph_layout)SPH_NLAYOUTS, &nsub, bytes));
        printf("invalid plan_out %d\n", (int)sph_plan_create(&cell, 1, &task, 1, 4, NULL));
    }
    return 0;
}

/* the loops through the per-task calls, `bundle` tasks per pack / launch / unpack */
static void per_task(const sph_plan *plan, const sph_store *store, int32_t ntask, int32_t bundle,
                     const sph_params *params)
{
    int32_t loop, t0;
    for (loop = 0; loop < 3; ++loop) {
        size_t pmax = 256, rmax = 256;
        void *pack = NULL, *res = NULL;
        /* buffers for the largest bundle */
        for (t0 = 0; t0 < ntask; t0 += bundle) {
            const int32_t t1 = t0 + bundle < ntask ? t0 + bundle : ntask;
            int64_t nslot = 0;
            size_t pb = 0, rb = 0;
            CHECK(sph_plan_buffer_bytes(plan, (sph_loop)loop, t0, t1, &nslot, &pb, &rb));
            if (pb > pmax) pmax = pb;
            if (rb > rmax) rmax = rb;
        }
        HIPCHECK(hipMalloc(&pack, pmax));
        HIPCHECK(hipMalloc(&res, rmax));
        CHECK(sph_zero_outputs(plan, (sph_loop)loop, store, NULL));
        for (t0 = 0; t0 < ntask; t0 += bundle) {
            const int32_t t1 = t0 + bundle < ntask ? t0 + bundle : ntask;
            CHECK(sph_pack(plan, (sph_loop)loop, store, t0, t1, pack, pmax, NULL));
            if (loop == SPH_DENSITY)
                CHECK(sph_density(plan, pack, pmax, t0, t1, params, res, rmax, NULL, NULL));
            else if (loop == SPH_GRADIENT)
                CHECK(sph_gradient(plan, pack, pmax, t0, t1, params, res, rmax, NULL, NULL));
            else
                CHECK(sph_force(plan, pack, pmax, t0, t1, params, res, rmax, NULL, NULL));
            CHECK(sph_unpack(plan, (sph_loop)loop, res, rmax, t0, t1, store, NULL));
        }
        HIPCHECK(hipDeviceSynchronize());
        HIPCHECK(hipFree(pack));
        HIPCHECK(hipFree(res));
    }
}

static int step(const char *in_path, const char *out_path, int32_t bundle)
{
    FILE *fin = fopen(in_path, "rb"), *fout;
    int64_t n;
    int32_t hdr[4], nsub = 0, s;
    size_t sub_bytes[SPH_MAX_SUB], ws_bytes = 0, i;
    sph_cell *cells;
    sph_task *tasks;
    sph_store store;
    sph_plan *plan = NULL;
    sph_params params;
    sph_tuning tuning;
    void *ws = NULL, *dbuf = NULL, *hbuf;
    static const sph_field in_fields[7] = {SPH_F_X, SPH_F_V, SPH_F_MASS, SPH_F_H, SPH_F_U, SPH_F_ALPHA_V,
                                           SPH_F_ALPHA_D};
    static const sph_field out_fields[9] = {SPH_F_RHO, SPH_F_RHO_DH, SPH_F_WCOUNT, SPH_F_DIV, SPH_F_ROT,
                                            SPH_F_LAP, SPH_F_VSIG, SPH_F_A, SPH_F_U_DT};
    if (!fin) {
        fprintf(stderr, "cannot open %s\n", in_path);
        return 1;
    }
    read_all(fin, &n, sizeof n);
    read_all(fin, hdr, sizeof hdr);
    if (n <= 0 || hdr[0] <= 0 || hdr[1] <= 0 || hdr[2] < 0 || hdr[2] >= SPH_NLAYOUTS) {
        fprintf(stderr, "bad header\n");
        return 1;
    }
    cells = (sph_cell *)host_alloc((size_t)hdr[0] * sizeof(sph_cell));
    tasks = (sph_task *)host_alloc((size_t)hdr[1] * sizeof(sph_task));
    read_all(fin, cells, (size_t)hdr[0] * sizeof(sph_cell));
    read_all(fin, tasks, (size_t)hdr[1] * sizeof(sph_task));

    /* the store: one device array per substruct, zero-filled */
    CHECK(sph_layout_info((sph_layout)hdr[2], &nsub, sub_bytes));
    memset(&store, 0, sizeof store);
    store.layout = hdr[2];
    store.nsub = nsub;
    store.n = n;
    for (s = 0; s < nsub; ++s) {
        HIPCHECK(hipMalloc(&store.sub[s], (size_t)n * sub_bytes[s]));
        HIPCHECK(hipMemset(store.sub[s], 0, (size_t)n * sub_bytes[s]));
    }
    /* input fields: host file -> staging device array -> setter */
    HIPCHECK(hipMalloc(&dbuf, (size_t)n * 24));
    hbuf = host_alloc((size_t)n * 24);
    for (i = 0; i < 7; ++i) {
        int32_t ncomp = 0, cb = 0;
        size_t bytes;
        CHECK(sph_field_info(in_fields[i], &ncomp, &cb));
        bytes = (size_t)n * (size_t)ncomp * (size_t)cb;
        read_all(fin, hbuf, bytes);
        HIPCHECK(hipMemcpy(dbuf, hbuf, bytes, hipMemcpyHostToDevice));
        CHECK(sph_store_put(&store, in_fields[i], dbuf, NULL));
    }
    fclose(fin);

    CHECK(sph_plan_create(cells, hdr[0], tasks, hdr[1], n, &plan));
    params.gamma_ad = 5.0f / 3.0f;
    params.beta_visc = 3.0f;
    params.balsara_eps = 1e-4f;
    params.pad = 0.0f;
    if (bundle > 0) {
        per_task(plan, &store, hdr[1], bundle, &params);
    } else {
        CHECK(sph_batched_ws_bytes(plan, &ws_bytes));
        HIPCHECK(hipMalloc(&ws, ws_bytes));
        sph_tuning_default(&tuning);
        CHECK(sph_step_batched(plan, &store, &params, &tuning, ws, ws_bytes, NULL));
        HIPCHECK(hipDeviceSynchronize());
    }

    fout = fopen(out_path, "wb");
    if (!fout) {
        fprintf(stderr, "cannot open %s\n", out_path);
        return 1;
    }
    for (i = 0; i < 9; ++i) {
        int32_t ncomp = 0, cb = 0;
        size_t bytes;
        CHECK(sph_field_info(out_fields[i], &ncomp, &cb));
        bytes = (size_t)n * (size_t)ncomp * (size_t)cb;
        CHECK(sph_store_get(&store, out_fields[i], dbuf, NULL));
        HIPCHECK(hipMemcpy(hbuf, dbuf, bytes, hipMemcpyDeviceToHost));
        if (fwrite(hbuf, 1, bytes, fout) != bytes) {
            fprintf(stderr, "short write\n");
            return 1;
        }
    }
    fclose(fout);
    sph_plan_destroy(plan);
    if (ws) HIPCHECK(hipFree(ws));
    HIPCHECK(hipFree(dbuf));
    for (s = 0; s < nsub; ++s) HIPCHECK(hipFree(store.sub[s]));
    free(hbuf);
    free(cells);
    free(tasks);
    printf("%s n=%lld cells=%d tasks=%d layout=%d ok\n", bundle > 0 ? "per_task" : "step", (long long)n, hdr[0],
           hdr[1], hdr[2]);
    return 0;
}

int main(int argc, char **argv)
{
    if (argc == 2 && strcmp(argv[1], "tables") == 0) return tables();
    if (argc == 4 && strcmp(argv[1], "step") == 0) return step(argv[2], argv[3], 0);
    if (argc == 5 && strcmp(argv[1], "per_task") == 0 && atoi(argv[4]) > 0)
        return step(argv[2], argv[3], (int32_t)atoi(argv[4]));
    fprintf(stderr, "usage: %s tables | step IN OUT | per_task IN OUT BUNDLE\n", argv[0]);
    return 2;
}
