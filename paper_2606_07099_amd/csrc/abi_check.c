/*
 * A plain C client of the C ABI in sable_pf.h: no Python, no torch.  Reads a
 * network and a batch of scenarios from a text file, builds a template,
 * solves, runs the adjoint of L = sum(|V|) + sum(theta) and prints the
 * results, so that a test can compare them with the oracle.
 *
 * Input (whitespace separated):
 *   n_bus n_branch batch precision(0 FP64, 1 mixed)
 *   bus_type[n_bus]
 *   from[n_branch] to[n_branch] r[n_branch] x[n_branch] bc[n_branch]
 *   pd[batch*n_bus] qd[batch*n_bus] pg[batch*n_bus] vset[batch*n_bus]
 * Output: one line per scenario: status iters, then vm[n_bus], va[n_bus],
 * g_pd[n_bus], g_qd[n_bus], g_pg[n_bus], g_vset[n_bus].
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "sable_pf.h"

static int fail(const char* what, int rc) {
  fprintf(stderr, "%s failed (%d): %s\n", what, rc, pf_last_error());
  return 1;
}

static int read_i(FILE* f, int32_t* a, int n) {
  for (int i = 0; i < n; ++i)
    if (fscanf(f, "%d", &a[i]) != 1) return 0;
  return 1;
}

static int read_d(FILE* f, double* a, int n) {
  for (int i = 0; i < n; ++i)
    if (fscanf(f, "%lf", &a[i]) != 1) return 0;
  return 1;
}

int main(int argc, char** argv) {
  if (argc != 2) { fprintf(stderr, "usage: abi_check input.txt\n"); return 2; }
  FILE* f = fopen(argv[1], "r");
  if (!f) { fprintf(stderr, "cannot open %s\n", argv[1]); return 2; }
  int n, m, batch, prec;
  if (fscanf(f, "%d %d %d %d", &n, &m, &batch, &prec) != 4 || n < 2 || m < 1 || batch < 1) return 2;
  const size_t nb = (size_t)batch * n;
  int32_t* bt = malloc(sizeof(int32_t) * n);
  int32_t *from = malloc(sizeof(int32_t) * m), *to = malloc(sizeof(int32_t) * m);
  double *r = malloc(sizeof(double) * m), *x = malloc(sizeof(double) * m), *bc = malloc(sizeof(double) * m);
  double* host[4];
  for (int k = 0; k < 4; ++k) host[k] = malloc(sizeof(double) * nb);
  if (!read_i(f, bt, n) || !read_i(f, from, m) || !read_i(f, to, m) || !read_d(f, r, m) ||
      !read_d(f, x, m) || !read_d(f, bc, m))
    return 2;
  for (int k = 0; k < 4; ++k)
    if (!read_d(f, host[k], (int)nb)) return 2;
  fclose(f);

  /* Y_bus through the library's pi-model helper */
  const int cap = 4 * m + n;
  int32_t* ip = malloc(sizeof(int32_t) * (n + 1));
  int32_t* ix = malloc(sizeof(int32_t) * cap);
  double *g = malloc(sizeof(double) * cap), *b = malloc(sizeof(double) * cap);
  int32_t nnz = 0;
  int rc = pf_ybus_from_branches(n, m, from, to, r, x, bc, ip, ix, g, b, cap, &nnz);
  if (rc != PF_OK) return fail("pf_ybus_from_branches", rc);

  pf_options opt;
  pf_default_options(&opt);
  opt.tol = 1e-10;
  opt.precision = prec ? PF_MIXED : PF_FP64;
  pf_template* tpl = NULL;
  rc = pf_template_build(n, bt, ip, ix, g, b, batch, &opt, &tpl);
  if (rc != PF_OK) return fail("pf_template_build", rc);

  /* device arrays: 4 inputs, vm va, 2 adjoint seeds, 4 gradients */
  double* d[12];
  for (int k = 0; k < 12; ++k)
    if (hipMalloc((void**)&d[k], sizeof(double) * nb) != hipSuccess) return fail("hipMalloc", -1);
  int32_t *d_it, *d_st;
  double* d_fn;
  if (hipMalloc((void**)&d_it, sizeof(int32_t) * batch) != hipSuccess ||
      hipMalloc((void**)&d_st, sizeof(int32_t) * batch) != hipSuccess ||
      hipMalloc((void**)&d_fn, sizeof(double) * batch) != hipSuccess)
    return fail("hipMalloc", -1);
  for (int k = 0; k < 4; ++k)
    if (hipMemcpy(d[k], host[k], sizeof(double) * nb, hipMemcpyHostToDevice) != hipSuccess)
      return fail("hipMemcpy", -1);
  rc = pf_solve_batch(tpl, d[0], d[1], d[2], d[3], d[4], d[5], d_it, d_st, d_fn, NULL);
  if (rc != PF_OK) return fail("pf_solve_batch", rc);
  /* dL/d|V| = dL/dtheta = 1 */
  double* ones = malloc(sizeof(double) * nb);
  for (size_t i = 0; i < nb; ++i) ones[i] = 1.0;
  if (hipMemcpy(d[6], ones, sizeof(double) * nb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d[7], ones, sizeof(double) * nb, hipMemcpyHostToDevice) != hipSuccess)
    return fail("hipMemcpy", -1);
  rc = pf_adjoint_batch(tpl, d[6], d[7], d[8], d[9], d[10], d[11], NULL);
  if (rc != PF_OK) return fail("pf_adjoint_batch", rc);
  if (hipDeviceSynchronize() != hipSuccess) return fail("hipDeviceSynchronize", -1);

  double* out[6];
  const int which[6] = {4, 5, 8, 9, 10, 11};
  for (int k = 0; k < 6; ++k) {
    out[k] = malloc(sizeof(double) * nb);
    if (hipMemcpy(out[k], d[which[k]], sizeof(double) * nb, hipMemcpyDeviceToHost) != hipSuccess)
      return fail("hipMemcpy", -1);
  }
  int32_t* it = malloc(sizeof(int32_t) * batch);
  int32_t* st = malloc(sizeof(int32_t) * batch);
  if (hipMemcpy(it, d_it, sizeof(int32_t) * batch, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(st, d_st, sizeof(int32_t) * batch, hipMemcpyDeviceToHost) != hipSuccess)
    return fail("hipMemcpy", -1);
  for (int s = 0; s < batch; ++s) {
    printf("%d %d", st[s], it[s]);
    for (int k = 0; k < 6; ++k)
      for (int i = 0; i < n; ++i) printf(" %.17g", out[k][(size_t)s * n + i]);
    printf("\n");
  }
  pf_template_destroy(tpl);
  for (int k = 0; k < 12; ++k) hipFree(d[k]);
  hipFree(d_it);
  hipFree(d_st);
  hipFree(d_fn);
  return 0;
}
