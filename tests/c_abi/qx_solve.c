/* A caller of libqx.so written against include/qx.h alone, with the HIP
 * runtime for device memory (no Python, no PyTorch): loads a gauge field and
 * a source from files, solves (m^2 - D_eo D_oe) x = b in mixed precision and
 * writes x.  Used by tests/test_gpu_c_abi.py.
 *
 *   qx_solve L0 L1 L2 L3 mass U.bin b.bin x.bin
 *
 * U.bin: complex128 [4][V][3][3]; b.bin, x.bin: complex128 [V/2][3]
 * (interleaved re, im doubles).  Prints "status iters updates relres" and
 * exits with the solver's status code (or 100 + a step number on an I/O or
 * HIP failure).
 */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "qx.h"

static int read_all(const char* path, void* dst, size_t bytes) {
  FILE* f = fopen(path, "rb");
  if (!f) return 0;
  const size_t n = fread(dst, 1, bytes, f);
  fclose(f);
  return n == bytes;
}

int main(int argc, char** argv) {
  if (argc != 9) {
    fprintf(stderr, "usage: %s L0 L1 L2 L3 mass U.bin b.bin x.bin\n", argv[0]);
    return 101;
  }
  const int32_t dims[4] = {atoi(argv[1]), atoi(argv[2]), atoi(argv[3]), atoi(argv[4])};
  const double mass = atof(argv[5]);
  qx_lattice_t* lat = NULL;
  if (qx_lattice_create(dims, 0, &lat) != QX_OK) {
    fprintf(stderr, "lattice: %s\n", qx_last_error());
    return 102;
  }
  const int64_t V = qx_lattice_volume(lat);
  const size_t u_bytes = (size_t)V * 4 * 9 * 16, f_bytes = (size_t)(V / 2) * 3 * 16;
  void* hU = malloc(u_bytes);
  void* hb = malloc(f_bytes);
  void* hx = malloc(f_bytes);
  if (!hU || !hb || !hx || !read_all(argv[6], hU, u_bytes) || !read_all(argv[7], hb, f_bytes)) {
    fprintf(stderr, "cannot read the inputs\n");
    return 103;
  }
  void *dU = NULL, *db = NULL, *dx = NULL, *p64 = NULL, *p32 = NULL, *ws = NULL;
  size_t g64_bytes = 0, g32_bytes = 0, ws_bytes = 0;
  qx_cg_params_t prm = {1e-10, 10000, QX_CG_MIXED_F32, 0.1, 0, 0, QX_ENGINE_AUTO};
  if (qx_gauge_bytes(lat, QX_PREC_F64, QX_RECON_18, &g64_bytes) != QX_OK ||
      qx_gauge_bytes(lat, QX_PREC_F32, QX_RECON_12, &g32_bytes) != QX_OK ||
      qx_cg_workspace_bytes(lat, &prm, 1, &ws_bytes) != QX_OK) {
    fprintf(stderr, "sizes: %s\n", qx_last_error());
    return 104;
  }
  if (hipMalloc(&dU, u_bytes) != hipSuccess || hipMalloc(&db, f_bytes) != hipSuccess ||
      hipMalloc(&dx, f_bytes) != hipSuccess || hipMalloc(&p64, g64_bytes) != hipSuccess ||
      hipMalloc(&p32, g32_bytes) != hipSuccess || hipMalloc(&ws, ws_bytes) != hipSuccess) {
    fprintf(stderr, "hipMalloc failed\n");
    return 105;
  }
  if (hipMemcpy(dU, hU, u_bytes, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(db, hb, f_bytes, hipMemcpyHostToDevice) != hipSuccess) {
    fprintf(stderr, "hipMemcpy failed\n");
    return 106;
  }
  qx_gauge_t *g64 = NULL, *g32 = NULL;
  if (qx_gauge_load(lat, dU, QX_PREC_F64, QX_RECON_18, p64, NULL, &g64) != QX_OK ||
      qx_gauge_load(lat, dU, QX_PREC_F32, QX_RECON_12, p32, NULL, &g32) != QX_OK) {
    fprintf(stderr, "gauge: %s\n", qx_last_error());
    return 107;
  }
  qx_cg_stats_t st;
  const int rc = qx_cg_solve(g64, g32, &prm, 1, &mass, db, dx, ws, ws_bytes, &st, NULL);
  if (rc != QX_OK) fprintf(stderr, "solve: %s\n", qx_last_error());
  if (hipMemcpy(hx, dx, f_bytes, hipMemcpyDeviceToHost) != hipSuccess) {
    fprintf(stderr, "hipMemcpy back failed\n");
    return 108;
  }
  FILE* f = fopen(argv[8], "wb");
  if (!f || fwrite(hx, 1, f_bytes, f) != f_bytes) {
    fprintf(stderr, "cannot write x\n");
    return 109;
  }
  fclose(f);
  printf("%d %d %d %.6e\n", st.status, st.iters, st.reliable_updates, st.true_rel_residual);
  qx_gauge_destroy(g64);
  qx_gauge_destroy(g32);
  qx_lattice_destroy(lat);
  hipFree(dU);
  hipFree(db);
  hipFree(dx);
  hipFree(p64);
  hipFree(p32);
  hipFree(ws);
  free(hU);
  free(hb);
  free(hx);
  return rc;
}
