/* A registration through the C-ABI alone: no Python, no torch and no HIP calls in this
 * program.  The images, masks and field stay in host memory (the library copies them), and
 * the device memory pool is the library's own.
 *
 * usage: c_register nx ny nz k params.bin target.f32 moving.f32 tmasks.u8 mmasks.u8 out.f32
 *   params.bin  one cgdir_params as raw bytes (its pointer fields null)
 *   *.f32       nx*ny*nz floats, x fastest;  *.u8: k masks of nx*ny*nz bytes each
 *   out.f32     the field, 3 planes (x, y, z components) of nx*ny*nz floats
 * Exit status 0 on success, else the library's error code is printed. */
#include <stdio.h>
#include <stdlib.h>

#include "cgdir.h"

static void *read_all(const char *path, size_t bytes)
{
    FILE *f = fopen(path, "rb");
    void *p = malloc(bytes ? bytes : 1);
    if (!f || !p || fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "cannot read %zu bytes from %s\n", bytes, path);
        exit(2);
    }
    fclose(f);
    return p;
}

int main(int argc, char **argv)
{
    if (argc != 11) {
        fprintf(stderr, "usage: %s nx ny nz k params.bin target moving tmasks mmasks out\n", argv[0]);
        return 2;
    }
    const int nx = atoi(argv[1]), ny = atoi(argv[2]), nz = atoi(argv[3]), k = atoi(argv[4]);
    if (nx < 1 || ny < 1 || nz < 1 || k < 0 || k > CGDIR_MAX_STRUCTS) return 2;
    const size_t n = (size_t)nx * ny * nz;
    cgdir_params *prm = (cgdir_params *)read_all(argv[5], sizeof(cgdir_params));
    float *target = (float *)read_all(argv[6], n * sizeof(float));
    float *moving = (float *)read_all(argv[7], n * sizeof(float));
    uint8_t *tm = (uint8_t *)read_all(argv[8], (size_t)k * n);
    uint8_t *mm = (uint8_t *)read_all(argv[9], (size_t)k * n);
    float *dvf = (float *)malloc(3 * n * sizeof(float));
    const uint8_t *tplanes[CGDIR_MAX_STRUCTS], *mplanes[CGDIR_MAX_STRUCTS];
    for (int i = 0; i < k; ++i) {
        tplanes[i] = tm + (size_t)i * n;
        mplanes[i] = mm + (size_t)i * n;
    }

    cgdir_ctx_desc desc = {0};
    desc.device = 0;
    desc.pool_bytes = (size_t)1 << 30;
    desc.max_slots = 1;
    cgdir_ctx *ctx = NULL;
    int rc = cgdir_create(&ctx, &desc);
    if (rc != CGDIR_OK) {
        fprintf(stderr, "cgdir_create: %s\n", cgdir_strerror(rc));
        return 1;
    }
    cgdir_volume t = {target, nx, ny, nz, CGDIR_HOST}, m = {moving, nx, ny, nz, CGDIR_HOST};
    cgdir_masks tmk = {k, tplanes, CGDIR_HOST}, mmk = {k, mplanes, CGDIR_HOST};
    rc = cgdir_register(ctx, &t, &m, k ? &tmk : NULL, k ? &mmk : NULL, prm, dvf, CGDIR_HOST);
    if (rc == CGDIR_OK) {
        FILE *f = fopen(argv[10], "wb");
        if (!f || fwrite(dvf, sizeof(float), 3 * n, f) != 3 * n) rc = -100;
        if (f) fclose(f);
    } else {
        fprintf(stderr, "cgdir_register: %s\n", cgdir_strerror(rc));
    }
    cgdir_destroy(ctx);
    free(prm);
    free(target);
    free(moving);
    free(tm);
    free(mm);
    free(dvf);
    return rc == CGDIR_OK ? 0 : 1;
}
