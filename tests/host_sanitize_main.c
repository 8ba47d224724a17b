/* Host-side checks of libslepian's C ABI under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_capi_host.py, host code
 * instrumented, no GPU needed): every entry point with null or out-of-domain
 * arguments, and the plan-file parser with malformed files (bad magic, a
 * truncated header, out-of-range fields, a short or long body, a non-finite
 * value).  Exits 0 when every call returns the expected status. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "slepian.h"

static int failures = 0;

#define EXPECT(call, want)                                                          \
  do {                                                                              \
    int got_ = (call);                                                              \
    if (got_ != (want)) {                                                           \
      fprintf(stderr, "%s:%d: %s returned %d, expected %d\n", __FILE__, __LINE__, #call, \
              got_, (int)(want));                                                   \
      ++failures;                                                                   \
    }                                                                               \
  } while (0)

/* plan-file header, as slepian_plan_save writes it */
typedef struct {
  char magic[8];
  int64_t N, K, win_lo, win_hi, u_l0, u_r;
  double W, eps, alpha;
  int32_t precision, pad;
  int64_t proj_off, proj_r, tik_off, tik_r;
  double lam_Km1, lam_K, eps_ach;
} header_t;

static void write_file(const char *path, const void *a, size_t na, const void *b, size_t nb) {
  FILE *f = fopen(path, "wb");
  if (!f) {
    perror(path);
    exit(2);
  }
  if (na) fwrite(a, 1, na, f);
  if (nb) fwrite(b, 1, nb, f);
  fclose(f);
}

static int load(const char *path) {
  slepian_plan_t p = NULL;
  int s = slepian_plan_load(path, -1, &p);
  if (s == SLEPIAN_OK) slepian_plan_destroy(p);
  else if (p != NULL) {
    fprintf(stderr, "failed load wrote a handle\n");
    ++failures;
  }
  return s;
}

int main(int argc, char **argv) {
  const char *dir = argc > 1 ? argv[1] : "/tmp";
  char path[4096];
  slepian_plan_t plan = NULL;
  slepian_plan_opts o;
  memset(&o, 0, sizeof(o));
  o.device = -1;
  size_t bytes = 0;

  /* domains */
  EXPECT(slepian_plan(1, 0.1, 1e-6, &plan), SLEPIAN_EINVAL);
  EXPECT(slepian_plan(64, 0.0, 1e-6, &plan), SLEPIAN_EINVAL);
  EXPECT(slepian_plan(64, 0.5, 1e-6, &plan), SLEPIAN_EINVAL);
  EXPECT(slepian_plan(64, NAN, 1e-6, &plan), SLEPIAN_EINVAL);
  EXPECT(slepian_plan(64, 0.1, 0.0, &plan), SLEPIAN_EINVAL);
  EXPECT(slepian_plan(64, 0.1, 0.5, &plan), SLEPIAN_EINVAL);
  EXPECT(slepian_plan(64, 0.1, INFINITY, &plan), SLEPIAN_EINVAL);
  EXPECT(slepian_plan(64, 0.1, 1e-6, NULL), SLEPIAN_EINVAL);
  EXPECT(slepian_plan((int64_t)1 << 40, 0.1, 1e-6, &plan), SLEPIAN_ENOTSUP);
  o.K = 64;
  EXPECT(slepian_plan_ex(64, 0.1, 1e-6, &o, &plan), SLEPIAN_EINVAL);
  o.K = 0;
  o.alpha = -1.0;
  EXPECT(slepian_plan_ex(64, 0.1, 1e-6, &o, &plan), SLEPIAN_EINVAL);
  o.alpha = 0.0;
  o.precision = 7;
  EXPECT(slepian_plan_ex(64, 0.1, 1e-6, &o, &plan), SLEPIAN_EINVAL);
  o.precision = 0;
  o.tune = 3;
  EXPECT(slepian_plan_ex(64, 0.1, 1e-6, &o, &plan), SLEPIAN_EINVAL);
  o.tune = 1;
  o.tune_batch = -5;
  EXPECT(slepian_plan_ex(64, 0.1, 1e-6, &o, &plan), SLEPIAN_EINVAL);
  o.tune = 0;
  o.tune_batch = 0;
  {
    int64_t Ns[3] = {100, 200, 1};
    double Ws[3] = {0.1, 0.1, 0.1}, Es[3] = {1e-6, 1e-6, 1e-6};
    slepian_plan_t hs[3] = {NULL, NULL, NULL};
    EXPECT(slepian_plan_batch(3, Ns, Ws, Es, NULL, hs), SLEPIAN_EINVAL);
    EXPECT(slepian_plan_batch(-1, Ns, Ws, Es, NULL, hs), SLEPIAN_EINVAL);
    EXPECT(slepian_plan_batch(0, NULL, NULL, NULL, NULL, NULL), SLEPIAN_OK);
  }

  /* null handles */
  EXPECT(slepian_plan_destroy(NULL), SLEPIAN_OK);
  EXPECT(slepian_workspace_size(NULL, SLEPIAN_OP_PROJECT, 4, &bytes), SLEPIAN_EINVAL);
  EXPECT(slepian_project(NULL, NULL, 0, NULL, 0, 1, NULL, 0, NULL), SLEPIAN_EINVAL);
  EXPECT(slepian_project_ex(NULL, 0, NULL, 0, NULL, 0, 1, NULL, 0, NULL), SLEPIAN_EINVAL);
  EXPECT(slepian_project_noalloc(NULL, NULL, 0, NULL, 0, 1, NULL), SLEPIAN_EINVAL);
  EXPECT(slepian_apply_b64(NULL, NULL, 0, NULL, 0, 1, NULL, 0, NULL), SLEPIAN_EINVAL);
  EXPECT(slepian_lsq(NULL, 0, 0.0, NULL, 0, NULL, 0, 1, 0.0, 0, NULL, 0, NULL, NULL), SLEPIAN_EINVAL);
  EXPECT(slepian_coeffs(NULL, NULL, 0, NULL, 0, 1, NULL, 0, NULL), SLEPIAN_EINVAL);
  EXPECT(slepian_plan_info_get(NULL, NULL), SLEPIAN_EINVAL);
  EXPECT(slepian_plan_save(NULL, "/tmp/never"), SLEPIAN_EINVAL);
  {
    double f[2] = {0.0, 0.25};
    slepian_bands_t bh = NULL;
    EXPECT(slepian_project_multiband(NULL, 2, f, NULL, 0, NULL, 0, 1, NULL, 0, NULL), SLEPIAN_EINVAL);
    EXPECT(slepian_bands_create(NULL, 2, f, &bh), SLEPIAN_EINVAL);
    EXPECT(slepian_bands_create(NULL, 2, f, NULL), SLEPIAN_EINVAL);
    EXPECT(slepian_bands_destroy(NULL), SLEPIAN_OK);
    EXPECT(slepian_bands_workspace_size(NULL, 4, &bytes), SLEPIAN_EINVAL);
    EXPECT(slepian_bands_span_workspace_size(NULL, 4, &bytes), SLEPIAN_EINVAL);
    EXPECT(slepian_project_bands(NULL, NULL, 0, NULL, 0, 1, NULL, 0, NULL), SLEPIAN_EINVAL);
    EXPECT(slepian_project_bands_span(NULL, NULL, 0, NULL, 0, 1, 0.0, 10, NULL, 0, NULL, NULL), SLEPIAN_EINVAL);
  }
  {
    slepian_factor_t fh = NULL;
    slepian_factor_info_t fi;
    EXPECT(slepian_factor_create(NULL, &fh), SLEPIAN_EINVAL);
    EXPECT(slepian_factor_create_ex(NULL, SLEPIAN_FACTOR_EIG, &fh), SLEPIAN_EINVAL);
    EXPECT(slepian_factor_create(NULL, NULL), SLEPIAN_EINVAL);
    EXPECT(slepian_factor_destroy(NULL), SLEPIAN_OK);
    EXPECT(slepian_factor_info(NULL, &fi), SLEPIAN_EINVAL);
    EXPECT(slepian_factor_mu(NULL, NULL, 0), SLEPIAN_EINVAL);
    EXPECT(slepian_factor_workspace_size(NULL, 4, &bytes), SLEPIAN_EINVAL);
    EXPECT(slepian_factor_compress(NULL, NULL, 0, NULL, 0, 1, NULL, 0, NULL), SLEPIAN_EINVAL);
    EXPECT(slepian_factor_recover(NULL, NULL, 0, NULL, 0, 1, NULL, 0, NULL), SLEPIAN_EINVAL);
  }
  {
    slepian_group_t gh = NULL;
    EXPECT(slepian_group_create(NULL, 0, NULL, &gh), SLEPIAN_EINVAL);
    EXPECT(slepian_group_destroy(NULL), SLEPIAN_OK);
    EXPECT(slepian_group_project(NULL, NULL, NULL, NULL), SLEPIAN_EINVAL);
    slepian_group_info_t gi;
    EXPECT(slepian_group_info(NULL, &gi), SLEPIAN_EINVAL);
  }
  for (int s = -12; s <= 0; ++s)
    if (slepian_status_string(s) == NULL || strlen(slepian_status_string(s)) == 0) {
      fprintf(stderr, "no status string for %d\n", s);
      ++failures;
    }

  /* plan files */
  EXPECT(slepian_plan_load(NULL, -1, &plan), SLEPIAN_EINVAL);
  EXPECT(slepian_plan_load("/nonexistent/plan.bin", -1, NULL), SLEPIAN_EINVAL);
  snprintf(path, sizeof(path), "%s/nonexistent_dir/plan.bin", dir);
  EXPECT(load(path), SLEPIAN_EIO);
  snprintf(path, sizeof(path), "%s/san_plan.bin", dir);
  write_file(path, "", 0, NULL, 0);
  EXPECT(load(path), SLEPIAN_EIO);
  {
    unsigned char junk[700];
    uint32_t z = 12345u;
    for (size_t i = 0; i < sizeof(junk); ++i) {
      z = z * 1664525u + 1013904223u;
      junk[i] = (unsigned char)(z >> 24);
    }
    write_file(path, junk, sizeof(junk), NULL, 0);
    EXPECT(load(path), SLEPIAN_EIO);
  }
  header_t h;
  memset(&h, 0, sizeof(h));
  memcpy(h.magic, "SLEPPLN1", 8);
  write_file(path, &h, sizeof(h) / 2, NULL, 0); /* truncated header */
  EXPECT(load(path), SLEPIAN_EIO);
  write_file(path, &h, sizeof(h), NULL, 0); /* N = 0 */
  EXPECT(load(path), SLEPIAN_EIO);
  /* a consistent small header: N = 64, window 0..15, U of 4 columns from l = 6 */
  h.N = 64;
  h.K = 13;
  h.W = 0.1;
  h.eps = 1e-6;
  h.win_lo = 0;
  h.win_hi = 15;
  h.u_l0 = 6;
  h.u_r = 4;
  h.proj_off = 0;
  h.proj_r = 4;
  h.tik_off = 0;
  h.tik_r = 0;
  h.lam_Km1 = 0.9;
  h.lam_K = 0.1;
  const size_t nbody = 16 + 2 * 4 + 64 * 4;
  double *body = (double *)calloc(nbody + 8, sizeof(double));
  for (size_t i = 0; i < nbody + 8; ++i) body[i] = 0.001 * (double)i;
  write_file(path, &h, sizeof(h), body, (nbody - 1) * sizeof(double)); /* one value short */
  EXPECT(load(path), SLEPIAN_EIO);
  write_file(path, &h, sizeof(h), body, (nbody + 8) * sizeof(double)); /* trailing data */
  EXPECT(load(path), SLEPIAN_EIO);
  body[20] = NAN;
  write_file(path, &h, sizeof(h), body, nbody * sizeof(double)); /* non-finite value */
  EXPECT(load(path), SLEPIAN_EIO);
  body[20] = 0.02;
  header_t hb = h;
  hb.u_l0 = 14; /* U's columns run past the window */
  write_file(path, &hb, sizeof(hb), body, nbody * sizeof(double));
  EXPECT(load(path), SLEPIAN_EIO);
  hb = h;
  hb.win_hi = 64; /* window past N */
  write_file(path, &hb, sizeof(hb), body, nbody * sizeof(double));
  EXPECT(load(path), SLEPIAN_EIO);
  hb = h;
  hb.proj_off = 2; /* set past U's columns */
  write_file(path, &hb, sizeof(hb), body, nbody * sizeof(double));
  EXPECT(load(path), SLEPIAN_EIO);
  hb = h;
  hb.u_r = (int64_t)1 << 40; /* a huge U must not be allocated */
  write_file(path, &hb, sizeof(hb), body, nbody * sizeof(double));
  EXPECT(load(path), SLEPIAN_EIO);
  hb = h;
  hb.eps = 0.7;
  write_file(path, &hb, sizeof(hb), body, nbody * sizeof(double));
  EXPECT(load(path), SLEPIAN_EIO);
  /* well-formed: parsed completely on the host, then the device step (no
     device here: a HIP error; with a device: a plan) */
  write_file(path, &h, sizeof(h), body, nbody * sizeof(double));
  {
    int s = load(path);
    if (s != SLEPIAN_EHIP && s != SLEPIAN_OK) {
      fprintf(stderr, "well-formed file: status %d\n", s);
      ++failures;
    }
  }
  free(body);
  remove(path);
  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("host checks passed\n");
  return 0;
}
