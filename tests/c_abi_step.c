/* A C99 caller of the step library, with no Python in between: it compiles a model from its
 * JSON file (rb_model_create_json), makes a batch, uploads the worlds' states and controls
 * from raw float32 files, advances them `steps` env steps with rb_step on the default stream,
 * and writes the final qpos, qvel and status words to a raw file.
 *
 *   c_abi_step MODEL.json N STEPS QPOS.f32 QVEL.f32 CTRL.f32 OUT.bin
 *
 * QPOS [N, nq], QVEL [N, nv] and CTRL [N, nu] are little-endian float32 (CTRL may be empty
 * when nu = 0); OUT holds qpos [N, nq] and qvel [N, nv] as float32, then status [N] as uint32.
 * Exit status 0 on success; otherwise the failing call and rb_last_error() go to stderr. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "rbstep.h"

static void* read_file(const char* path, size_t* size) {
    FILE* f = fopen(path, "rb");
    if (!f) return NULL;
    fseek(f, 0, SEEK_END);
    long n = ftell(f);
    fseek(f, 0, SEEK_SET);
    char* buf = (char*)malloc((size_t)n + 1);
    if (buf && n > 0 && fread(buf, 1, (size_t)n, f) != (size_t)n) {
        free(buf);
        buf = NULL;
    }
    fclose(f);
    if (buf) buf[n] = 0;
    *size = (size_t)n;
    return buf;
}

#define CHECK_RB(call)                                                              \
    do {                                                                            \
        int rc_ = (call);                                                           \
        if (rc_ != RB_OK) {                                                         \
            fprintf(stderr, "%s failed (%d): %s\n", #call, rc_, rb_last_error());  \
            return 1;                                                               \
        }                                                                           \
    } while (0)
#define CHECK_HIP(call)                                                             \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) {                                                     \
            fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));      \
            return 1;                                                               \
        }                                                                           \
    } while (0)

int main(int argc, char** argv) {
    if (argc != 8) {
        fprintf(stderr, "usage: %s MODEL.json N STEPS QPOS.f32 QVEL.f32 CTRL.f32 OUT.bin\n", argv[0]);
        return 2;
    }
    const int n = atoi(argv[2]), steps = atoi(argv[3]);
    size_t sz = 0, sq = 0, sv = 0, su = 0;
    char* json = (char*)read_file(argv[1], &sz);
    float* q = (float*)read_file(argv[4], &sq);
    float* v = (float*)read_file(argv[5], &sv);
    float* u = (float*)read_file(argv[6], &su);
    if (!json || !q || !v || !u || n <= 0 || steps < 0) {
        fprintf(stderr, "bad arguments or unreadable files\n");
        return 2;
    }
    rb_model* model = NULL;
    rb_batch* batch = NULL;
    rb_model_info info;
    CHECK_RB(rb_model_create_json(json, &model));
    CHECK_RB(rb_model_info_get(model, &info));
    if (sq != sizeof(float) * (size_t)n * info.nq || sv != sizeof(float) * (size_t)n * info.nv ||
        su != sizeof(float) * (size_t)n * info.nu) {
        fprintf(stderr, "input sizes do not match the model (nq %d, nv %d, nu %d)\n", info.nq, info.nv, info.nu);
        return 2;
    }
    CHECK_RB(rb_batch_create(model, n, 0, &batch));
    float *dq = NULL, *dv = NULL, *du = NULL;
    uint32_t* dst = NULL;
    CHECK_HIP(hipMalloc((void**)&dq, sq));
    CHECK_HIP(hipMalloc((void**)&dv, sv));
    if (info.nu > 0) CHECK_HIP(hipMalloc((void**)&du, su));
    CHECK_HIP(hipMalloc((void**)&dst, sizeof(uint32_t) * (size_t)n));
    CHECK_HIP(hipMemcpy(dq, q, sq, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(dv, v, sv, hipMemcpyHostToDevice));
    if (du) CHECK_HIP(hipMemcpy(du, u, su, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemset(dst, 0, sizeof(uint32_t) * (size_t)n));
    for (int s = 0; s < steps; s++) CHECK_RB(rb_step(batch, n, du, dq, dv, NULL, dst, NULL));
    CHECK_HIP(hipDeviceSynchronize());
    uint32_t* st = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
    if (!st) return 1;
    CHECK_HIP(hipMemcpy(q, dq, sq, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(v, dv, sv, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(st, dst, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToHost));
    FILE* out = fopen(argv[7], "wb");
    if (!out || fwrite(q, 1, sq, out) != sq || fwrite(v, 1, sv, out) != sv ||
        fwrite(st, sizeof(uint32_t), (size_t)n, out) != (size_t)n) {
        fprintf(stderr, "cannot write %s\n", argv[7]);
        return 1;
    }
    fclose(out);
    hipFree(dq);
    hipFree(dv);
    if (du) hipFree(du);
    hipFree(dst);
    rb_batch_destroy(batch);
    rb_model_destroy(model);
    free(json);
    free(q);
    free(v);
    free(u);
    free(st);
    printf("c_abi_step: %d worlds x %d env steps of %s\n", n, steps, argv[1]);
    return 0;
}
