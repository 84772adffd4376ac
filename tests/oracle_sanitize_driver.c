/* oracle_sanitize_driver.c -- runs every entry point of the FP64 oracle on inputs
 * read from files, so that the oracle can be built and exercised under
 * AddressSanitizer + UndefinedBehaviorSanitizer or ThreadSanitizer (test
 * infrastructure: only tests/test_oracle_sanitize.py builds and runs it).
 *
 * usage: oracle_sanitize_driver DIR B J T NTHREADS
 * reads  DIR/{n,adj,fixed,motor,x0}.bin (the links_batch layout, x0 as double)
 * writes DIR/{order,n_dyads,depth,st_order}.bin         links_ref_solve_order
 *        DIR/{status,fail,path,pos_all,margins}.bin     continuity rule
 *        DIR/{status_o,fail_o}.bin                      orientation rule
 *        DIR/{norm_pca,xf_pca,norm_diam,xf_diam}.bin    both normalisations of every path row
 *        DIR/{cur_flags,cur_var,cur_keep}.bin          curation of the diameter rows
 * Exit status 0 when every call returned 0. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "links_ref.h"

static void* read_all(const char* dir, const char* name, size_t bytes) {
  char p[4096];
  snprintf(p, sizeof(p), "%s/%s.bin", dir, name);
  FILE* f = fopen(p, "rb");
  if (!f) {
    fprintf(stderr, "cannot open %s\n", p);
    exit(2);
  }
  void* buf = malloc(bytes ? bytes : 1);
  if (!buf || fread(buf, 1, bytes, f) != bytes) {
    fprintf(stderr, "short read of %s\n", p);
    exit(2);
  }
  fclose(f);
  return buf;
}

static void write_all(const char* dir, const char* name, const void* buf, size_t bytes) {
  char p[4096];
  snprintf(p, sizeof(p), "%s/%s.bin", dir, name);
  FILE* f = fopen(p, "wb");
  if (!f || fwrite(buf, 1, bytes, f) != bytes) {
    fprintf(stderr, "cannot write %s\n", p);
    exit(2);
  }
  fclose(f);
}

int main(int argc, char** argv) {
  if (argc != 6) {
    fprintf(stderr, "usage: %s DIR B J T NTHREADS\n", argv[0]);
    return 2;
  }
  const char* dir = argv[1];
  const int32_t B = atoi(argv[2]), J = atoi(argv[3]), T = atoi(argv[4]), nth = atoi(argv[5]);
  uint8_t* n = read_all(dir, "n", (size_t)B);
  uint32_t* adj = read_all(dir, "adj", (size_t)B * J * 4);
  uint32_t* fixed = read_all(dir, "fixed", (size_t)B * 4);
  uint8_t* motor = read_all(dir, "motor", (size_t)B * 2);
  double* x0 = read_all(dir, "x0", (size_t)B * J * 2 * 8);
  int rc = 0;

  int8_t* order = malloc((size_t)B * J * 3 + 1);
  uint8_t *nd = malloc(B + 1), *dp = malloc(B + 1), *so = malloc(B + 1);
  rc |= links_ref_solve_order(B, J, n, adj, fixed, motor, order, nd, dp, so);
  write_all(dir, "order", order, (size_t)B * J * 3);
  write_all(dir, "n_dyads", nd, B);
  write_all(dir, "depth", dp, B);
  write_all(dir, "st_order", so, B);

  uint8_t* st = malloc(B + 1);
  int16_t* fs = malloc((size_t)B * 2 + 2);
  double* path = malloc((size_t)B * T * 2 * 8 + 8);
  double* all = malloc((size_t)B * T * J * 2 * 8 + 8);
  double* mg = malloc((size_t)B * 4 * 8 + 8);
  rc |= links_ref_simulate_branch(B, J, n, adj, fixed, motor, x0, T, -1, 1e-4, st, fs, path, all, mg, nth,
                                  LREF_BRANCH_CONTINUITY);
  write_all(dir, "status", st, B);
  write_all(dir, "fail", fs, (size_t)B * 2);
  write_all(dir, "path", path, (size_t)B * T * 2 * 8);
  write_all(dir, "pos_all", all, (size_t)B * T * J * 2 * 8);
  write_all(dir, "margins", mg, (size_t)B * 4 * 8);

  uint8_t* st_o = malloc(B + 1);
  int16_t* fs_o = malloc((size_t)B * 2 + 2);
  rc |= links_ref_simulate_branch(B, J, n, adj, fixed, motor, x0, T, -1, 1e-4, st_o, fs_o, NULL, NULL, NULL, nth,
                                  LREF_BRANCH_ORIENTATION);
  write_all(dir, "status_o", st_o, B);
  write_all(dir, "fail_o", fs_o, (size_t)B * 2);

  double* norm = malloc((size_t)B * T * 2 * 8 + 8);
  double* xf = malloc((size_t)B * 5 * 8 + 8);
  rc |= links_ref_normalize_paths(path, B, T, LREF_NORM_PCA, norm, xf);
  write_all(dir, "norm_pca", norm, (size_t)B * T * 2 * 8);
  write_all(dir, "xf_pca", xf, (size_t)B * 5 * 8);
  rc |= links_ref_normalize_paths(path, B, T, LREF_NORM_DIAMETER, norm, xf);
  write_all(dir, "norm_diam", norm, (size_t)B * T * 2 * 8);
  write_all(dir, "xf_diam", xf, (size_t)B * 5 * 8);

  uint8_t* cf = malloc(B + 1);
  double* cv = malloc((size_t)B * 8 + 8);
  uint32_t* ck = malloc((size_t)B * 4 + 4);
  rc |= links_ref_curate(J, n, adj, fixed, motor, -1, NULL, B, norm, T, 5e-4, cf, cv, ck);
  write_all(dir, "cur_flags", cf, B);
  write_all(dir, "cur_var", cv, (size_t)B * 8);
  write_all(dir, "cur_keep", ck, (size_t)B * 4);

  free(n), free(adj), free(fixed), free(motor), free(x0), free(order), free(nd), free(dp), free(so);
  free(st), free(fs), free(path), free(all), free(mg), free(st_o), free(fs_o), free(norm), free(xf);
  free(cf), free(cv), free(ck);
  return rc != 0;
}
