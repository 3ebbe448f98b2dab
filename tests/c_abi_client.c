/*
 * A plain C99 client of the t-SGNE library, for the tests: it reads a graph
 * (canonical symmetric CSR), an embedding and an initial layout from a
 * binary file, moves them to the device with the HIP runtime, runs
 * tsgne_build_P, tsgne_run and tsgne_kl through the C-ABI only, and writes
 * the final layout and KL.  It also checks an error path (n = 0 is refused
 * with TSGNE_E_INVAL and a message).
 *
 * Input : int32 n, int64 nnz, int32 d, int32 n_iter, int32 exaggeration_iters,
 *         float perplexity, int32 row_ptr[n+1], int32 col[nnz],
 *         float X[n*d], float Y0[n*2]
 * Output: double kl, float Y[n*2]
 * Usage : c_abi_client <input> <output>; exit status 0 on success.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "tsgne.h"

static int fail_tsgne(const char* what, tsgne_status st) {
  fprintf(stderr, "%s: %s: %s\n", what, tsgne_status_string(st), tsgne_last_error());
  return 1;
}

static int fail_hip(const char* what, hipError_t e) {
  fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
  return 1;
}

static int read_all(FILE* f, void* p, size_t bytes) { return bytes == 0 || fread(p, 1, bytes, f) == bytes; }

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s <input> <output>\n", argv[0]);
    return 2;
  }
  FILE* in = fopen(argv[1], "rb");
  if (!in) return 2;
  int32_t n = 0, d = 0, n_iter = 0, t_ee = 0;
  int64_t nnz = 0;
  float perplexity = 0.f;
  if (!read_all(in, &n, 4) || !read_all(in, &nnz, 8) || !read_all(in, &d, 4) || !read_all(in, &n_iter, 4) ||
      !read_all(in, &t_ee, 4) || !read_all(in, &perplexity, 4) || n < 1 || nnz < 0 || d < 1)
    return 2;
  int32_t* row_ptr = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  int32_t* col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  float* X = (float*)malloc(sizeof(float) * (size_t)n * d);
  float* Y = (float*)malloc(sizeof(float) * (size_t)n * 2);
  if (!row_ptr || !col || !X || !Y) return 2;
  if (!read_all(in, row_ptr, sizeof(int32_t) * ((size_t)n + 1)) || !read_all(in, col, sizeof(int32_t) * (size_t)nnz) ||
      !read_all(in, X, sizeof(float) * (size_t)n * d) || !read_all(in, Y, sizeof(float) * (size_t)n * 2))
    return 2;
  fclose(in);

  /* an argument error is refused on the host, with a message */
  tsgne_graph* bad = NULL;
  tsgne_status st = tsgne_build_P(0, 0, row_ptr, col, X, d, perplexity, NULL, &bad);
  if (st != TSGNE_E_INVAL || bad != NULL || tsgne_last_error()[0] == '\0') {
    fprintf(stderr, "n = 0 was not refused as expected\n");
    return 1;
  }

  int32_t *row_ptr_d = NULL, *col_d = NULL;
  float *X_d = NULL, *Y_d = NULL;
  hipError_t e;
  if ((e = hipMalloc((void**)&row_ptr_d, sizeof(int32_t) * ((size_t)n + 1))) != hipSuccess) return fail_hip("hipMalloc", e);
  if ((e = hipMalloc((void**)&col_d, sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1))) != hipSuccess) return fail_hip("hipMalloc", e);
  if ((e = hipMalloc((void**)&X_d, sizeof(float) * (size_t)n * d)) != hipSuccess) return fail_hip("hipMalloc", e);
  if ((e = hipMalloc((void**)&Y_d, sizeof(float) * (size_t)n * 2)) != hipSuccess) return fail_hip("hipMalloc", e);
  if ((e = hipMemcpy(row_ptr_d, row_ptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice)) != hipSuccess)
    return fail_hip("copy row_ptr", e);
  if (nnz > 0 && (e = hipMemcpy(col_d, col, sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice)) != hipSuccess)
    return fail_hip("copy col", e);
  if ((e = hipMemcpy(X_d, X, sizeof(float) * (size_t)n * d, hipMemcpyHostToDevice)) != hipSuccess) return fail_hip("copy X", e);
  if ((e = hipMemcpy(Y_d, Y, sizeof(float) * (size_t)n * 2, hipMemcpyHostToDevice)) != hipSuccess) return fail_hip("copy Y0", e);

  tsgne_graph* g = NULL;
  if ((st = tsgne_build_P(n, nnz, row_ptr_d, col_d, X_d, d, perplexity, NULL, &g)) != TSGNE_OK)
    return fail_tsgne("tsgne_build_P", st);
  tsgne_params p;
  tsgne_params_default(&p);
  p.exaggeration_iters = t_ee;
  if ((st = tsgne_run(g, Y_d, n_iter, &p, NULL, NULL)) != TSGNE_OK) return fail_tsgne("tsgne_run", st);
  double kl = 0.0;
  if ((st = tsgne_kl(g, Y_d, &kl, NULL)) != TSGNE_OK) return fail_tsgne("tsgne_kl", st);
  if ((e = hipMemcpy(Y, Y_d, sizeof(float) * (size_t)n * 2, hipMemcpyDeviceToHost)) != hipSuccess) return fail_hip("copy Y", e);
  tsgne_graph_free(g);
  hipFree(row_ptr_d);
  hipFree(col_d);
  hipFree(X_d);
  hipFree(Y_d);

  FILE* out = fopen(argv[2], "wb");
  if (!out || fwrite(&kl, 8, 1, out) != 1 || fwrite(Y, sizeof(float), (size_t)n * 2, out) != (size_t)n * 2) return 2;
  fclose(out);
  free(row_ptr);
  free(col);
  free(X);
  free(Y);
  return 0;
}
