/*
 * Plain-C client of the ICNNM C ABI: no Python and no PyTorch on the path; device
 * memory comes from hipMalloc. Reads a problem from raw files, solves it and writes
 * the completed tensor.
 *
 *   solve_c DIR m1 m2 m3 k1 k2 k3 iters precision
 *
 * DIR holds M.f32 (m1*m2*m3 float32, C order), mask.u8 (uint8, 1 = observed) and
 * V.f32 (k*k float32, row-major, k = k1*k2*k3); the result goes to DIR/L.f32 and
 * one line "iters r_primal r_change objective" to stdout. precision: 0 FP32,
 * 1 BF16, 2 FP16. Exit status 0 on success, 1 on a usage or I/O error, 2 on a
 * HIP error, 3 on an ICNNM error (its message on stderr).
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "icnnm.h"

static void* read_file(const char* dir, const char* name, size_t bytes) {
  char path[4096];
  snprintf(path, sizeof path, "%s/%s", dir, name);
  FILE* f = fopen(path, "rb");
  if (!f) return NULL;
  void* buf = malloc(bytes);
  size_t got = buf ? fread(buf, 1, bytes, f) : 0;
  fclose(f);
  if (got != bytes) {
    free(buf);
    return NULL;
  }
  return buf;
}

int main(int argc, char** argv) {
  if (argc != 10) {
    fprintf(stderr, "usage: %s DIR m1 m2 m3 k1 k2 k3 iters precision\n", argv[0]);
    return 1;
  }
  icnnm_shape shape;
  shape.ndim = 3;
  for (int d = 0; d < 3; ++d) {
    shape.m[d] = atoll(argv[2 + d]);
    shape.kdim[d] = atoll(argv[5 + d]);
  }
  const size_t n = (size_t)(shape.m[0] * shape.m[1] * shape.m[2]);
  const size_t k = (size_t)(shape.kdim[0] * shape.kdim[1] * shape.kdim[2]);
  float* M = (float*)read_file(argv[1], "M.f32", n * sizeof(float));
  unsigned char* mask = (unsigned char*)read_file(argv[1], "mask.u8", n);
  float* V = (float*)read_file(argv[1], "V.f32", k * k * sizeof(float));
  if (!M || !mask || !V) {
    fprintf(stderr, "cannot read M.f32, mask.u8 or V.f32 in %s\n", argv[1]);
    return 1;
  }
  float *dM = NULL, *dV = NULL, *dL = NULL;
  unsigned char* dmask = NULL;
  if (hipMalloc((void**)&dM, n * sizeof(float)) != hipSuccess || hipMalloc((void**)&dmask, n) != hipSuccess ||
      hipMalloc((void**)&dV, k * k * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&dL, n * sizeof(float)) != hipSuccess ||
      hipMemcpy(dM, M, n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dmask, mask, n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dV, V, k * k * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    fprintf(stderr, "HIP allocation or copy failed\n");
    return 2;
  }
  icnnm_ctx* ctx = NULL;
  icnnm_status rc = icnnm_create(0, 0, &ctx);
  if (rc != ICNNM_OK) {
    fprintf(stderr, "icnnm_create: status %d\n", (int)rc);
    return 3;
  }
  icnnm_params p;
  icnnm_params_default(&p);
  p.max_iter = atoi(argv[8]);
  p.precision = atoi(argv[9]);
  icnnm_info info;
  rc = icnnm_solve(ctx, &shape, dM, dmask, dV, &p, dL, &info, NULL);
  if (rc != ICNNM_OK) {
    fprintf(stderr, "icnnm_solve: status %d: %s\n", (int)rc, icnnm_last_error(ctx));
    icnnm_destroy(ctx);
    return 3;
  }
  float* L = (float*)malloc(n * sizeof(float));
  if (!L || hipMemcpy(L, dL, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) {
    fprintf(stderr, "HIP copy of the result failed\n");
    return 2;
  }
  char path[4096];
  snprintf(path, sizeof path, "%s/L.f32", argv[1]);
  FILE* f = fopen(path, "wb");
  if (!f || fwrite(L, sizeof(float), n, f) != n) {
    fprintf(stderr, "cannot write %s\n", path);
    return 1;
  }
  fclose(f);
  printf("%d %.9e %.9e %.9e\n", info.iters, info.r_primal, info.r_change, info.objective);
  icnnm_destroy(ctx);
  (void)hipFree(dM);
  (void)hipFree(dmask);
  (void)hipFree(dV);
  (void)hipFree(dL);
  free(M);
  free(mask);
  free(V);
  free(L);
  return 0;
}
