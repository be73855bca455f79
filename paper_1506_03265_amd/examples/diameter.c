/*
 * Diameter estimate of a weighted grid through the C ABI alone (no Python):
 * upload a CSR, validate and pack it, decompose it (CLUSTER), build the
 * weighted quotient graph and estimate the diameter.
 *
 * Build (from the repository root, after building libcldiam.so):
 *   gcc -std=c11 -O2 -D__HIP_PLATFORM_AMD__ -I include -I /opt/rocm/include \
 *       paper_1506_03265_amd/examples/diameter.c -o diameter \
 *       -L paper_1506_03265_amd -lcldiam -L /opt/rocm/lib -lamdhip64 \
 *       -Wl,-rpath,$PWD/paper_1506_03265_amd -Wl,-rpath,/opt/rocm/lib
 *   ./diameter 512 768
 *
 * The caller owns every device buffer and workspace; the library allocates no
 * device memory.
 */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "cldiam.h"

#define HIP_OK(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) {                                                          \
      fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));                     \
      exit(1);                                                                       \
    }                                                                                \
  } while (0)

#define CLD_OK(call)                                                                 \
  do {                                                                               \
    int s_ = (call);                                                                 \
    if (s_ != CLDIAM_OK) {                                                           \
      fprintf(stderr, "%s: %s (%s)\n", #call, cldiam_strerror(s_), cldiam_last_error()); \
      exit(1);                                                                       \
    }                                                                                \
  } while (0)

static void *dalloc(size_t bytes) {
  void *p = NULL;
  HIP_OK(hipMalloc(&p, bytes ? bytes : 1));
  return p;
}

/* rows x cols 4-neighbour grid; edge weight from a small integer hash of the
 * unordered pair, in [1, 1000], so both arcs of an edge carry the same weight */
static uint32_t edge_weight(int64_t a, int64_t b) {
  uint64_t x = (uint64_t)(a < b ? a : b) * 0x9E3779B97F4A7C15ull ^ (uint64_t)(a < b ? b : a);
  x ^= x >> 31;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 29;
  return 1u + (uint32_t)(x % 1000u);
}

int main(int argc, char **argv) {
  const int32_t rows = argc > 1 ? atoi(argv[1]) : 256, cols = argc > 2 ? atoi(argv[2]) : 256;
  const int32_t n = rows * cols;
  int64_t *rp = malloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t *col = malloc(sizeof(int32_t) * 4 * (size_t)n);
  uint32_t *w = malloc(sizeof(uint32_t) * 4 * (size_t)n);
  int64_t m = 0;
  for (int32_t v = 0; v < n; ++v) {   /* neighbours in ascending id: up, left, right, down */
    const int32_t r = v / cols, c = v % cols;
    rp[v] = m;
    const int32_t nb[4] = {r > 0 ? v - cols : -1, c > 0 ? v - 1 : -1, c + 1 < cols ? v + 1 : -1,
                           r + 1 < rows ? v + cols : -1};
    for (int k = 0; k < 4; ++k)
      if (nb[k] >= 0) { col[m] = nb[k]; w[m] = edge_weight(v, nb[k]); ++m; }
  }
  rp[n] = m;

  hipStream_t stream;
  HIP_OK(hipStreamCreate(&stream));
  int64_t *d_rp = dalloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t *d_col = dalloc(sizeof(int32_t) * (size_t)m);
  uint32_t *d_w = dalloc(sizeof(uint32_t) * (size_t)m);
  uint64_t *d_arcs = dalloc(sizeof(uint64_t) * (size_t)m);
  HIP_OK(hipMemcpy(d_rp, rp, sizeof(int64_t) * ((size_t)n + 1), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(d_col, col, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(d_w, w, sizeof(uint32_t) * (size_t)m, hipMemcpyHostToDevice));

  /* ingest: validation and weight-sorted packed arcs */
  cldiam_csr csr = {n, 0, m, d_rp, d_col, d_w};
  uint64_t wsum = 0;
  size_t wsb = cldiam_load_csr_workspace_size(n, m);
  void *ws = dalloc(wsb);
  CLD_OK(cldiam_load_csr(&csr, d_arcs, &wsum, ws, wsb, stream));
  HIP_OK(hipFree(ws));

  /* decomposition: CLUSTER(G, tau = 1), seed 1, default initial Delta */
  int32_t *d_cluster = dalloc(sizeof(int32_t) * (size_t)n);
  uint64_t *d_D = dalloc(sizeof(uint64_t) * (size_t)n);
  cldiam_graph gd = {n, 0, m, d_rp, d_arcs, wsum, {1, 0, 1, CLDIAM_VARIANT_FIXPOINT, 0}, d_cluster, d_D};
  cldiam_stats st;
  wsb = cldiam_decompose_workspace_size(n, 1);
  ws = dalloc(wsb);
  CLD_OK(cldiam_decompose(&gd, &st, CLDIAM_DRIVER_AUTO, NULL, ws, wsb, stream));
  HIP_OK(hipFree(ws));

  /* weighted quotient graph and the estimate */
  int32_t *d_qcenter = dalloc(sizeof(int32_t) * (size_t)n);
  int64_t *d_qrp = dalloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t *d_qcol = dalloc(sizeof(int32_t) * (size_t)m);
  uint64_t *d_qw = dalloc(sizeof(uint64_t) * (size_t)m);
  int32_t k = 0;
  int64_t qm = 0;
  wsb = cldiam_quotient_workspace_size(n, m);
  ws = dalloc(wsb);
  CLD_OK(cldiam_build_quotient(n, m, d_rp, d_arcs, d_cluster, d_D, d_qcenter, d_qrp, d_qcol, d_qw, &k, &qm, ws, wsb,
                               stream));
  HIP_OK(hipFree(ws));
  uint64_t phi_gc = 0, phi_approx = 0;
  wsb = cldiam_estimate_workspace_size(k, qm);
  ws = dalloc(wsb);
  CLD_OK(cldiam_estimate_diameter(k, qm, d_qrp, d_qcol, d_qw, st.radius, &phi_gc, &phi_approx, ws, wsb, stream));
  HIP_OK(hipFree(ws));

  printf("%d x %d grid: n=%d m=%lld arcs; %d clusters, radius %llu, %d stages; "
         "Phi(G_C) = %llu, estimate %llu (%.3f ms of decomposition)\n",
         rows, cols, n, (long long)m, k, (unsigned long long)st.radius, st.stages, (unsigned long long)phi_gc,
         (unsigned long long)phi_approx, st.kernel_ms);

  HIP_OK(hipFree(d_rp)); HIP_OK(hipFree(d_col)); HIP_OK(hipFree(d_w)); HIP_OK(hipFree(d_arcs));
  HIP_OK(hipFree(d_cluster)); HIP_OK(hipFree(d_D)); HIP_OK(hipFree(d_qcenter)); HIP_OK(hipFree(d_qrp));
  HIP_OK(hipFree(d_qcol)); HIP_OK(hipFree(d_qw));
  HIP_OK(hipStreamDestroy(stream));
  free(rp); free(col); free(w);
  return 0;
}
