/*
 * rtbte from plain C: read one problem and a state from a directory of raw
 * little-endian arrays, build a context, evaluate the right-hand side on the
 * GPU and write it back.  Shows the C ABI without any Python or PyTorch: the
 * caller owns the device buffers (hipMalloc) and the library works on them.
 *
 *   example_rhs <dir> [t_out]
 *
 * <dir>/meta.txt: n_el n_ph n_k_total n_q_total n_eph n_pp sigma_eph sigma_pp
 *                 nsigma hw_cut
 * <dir>/{eps,hw,eph_g2,pp_v2,y}.f64 and {eph_row,eph_partner,eph_phonon,
 * pp_row,pp_a,pp_b}.i32: the arrays of rtbte_problem and the state y.
 * Writes <dir>/ydot.f64 and prints the channel counts.  With t_out (fs), it
 * then advances y from t = 0 to t_out with the adaptive Zonneveld ERK
 * (default options, starting step chosen by the library) and writes
 * <dir>/y_out.f64 and a second line: accepted steps, rejected steps.  Exit
 * status 0 on success, 1 with a message on any failure.
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "rtbte.h"

static void *read_file(const char *dir, const char *name, size_t elem, int64_t n) {
  char path[4096];
  snprintf(path, sizeof path, "%s/%s", dir, name);
  void *buf = malloc(n > 0 ? (size_t)n * elem : 1);
  FILE *f = fopen(path, "rb");
  if (!buf || !f || (n > 0 && fread(buf, elem, (size_t)n, f) != (size_t)n)) {
    fprintf(stderr, "cannot read %s\n", path);
    exit(1);
  }
  fclose(f);
  return buf;
}

int main(int argc, char **argv) {
  if (argc != 2 && argc != 3) {
    fprintf(stderr, "usage: %s <dir> [t_out]\n", argv[0]);
    return 1;
  }
  const char *dir = argv[1];
  char path[4096];
  snprintf(path, sizeof path, "%s/meta.txt", dir);
  FILE *m = fopen(path, "r");
  rtbte_problem p;
  memset(&p, 0, sizeof p);
  long long n_eph = 0, n_pp = 0;
  if (!m || fscanf(m, "%d %d %d %d %lld %lld %lf %lf %lf %lf", &p.n_el, &p.n_ph, &p.n_k_total, &p.n_q_total,
                   &n_eph, &n_pp, &p.sigma_eph, &p.sigma_pp, &p.nsigma, &p.hw_cut) != 10) {
    fprintf(stderr, "cannot read %s\n", path);
    return 1;
  }
  fclose(m);
  p.n_eph = n_eph;
  p.n_pp = n_pp;
  p.eps = read_file(dir, "eps.f64", 8, p.n_el);
  p.hw = read_file(dir, "hw.f64", 8, p.n_ph);
  p.eph_row = read_file(dir, "eph_row.i32", 4, n_eph);
  p.eph_partner = read_file(dir, "eph_partner.i32", 4, n_eph);
  p.eph_phonon = read_file(dir, "eph_phonon.i32", 4, n_eph);
  p.eph_g2 = read_file(dir, "eph_g2.f64", 8, n_eph);
  p.pp_row = read_file(dir, "pp_row.i32", 4, n_pp);
  p.pp_a = read_file(dir, "pp_a.i32", 4, n_pp);
  p.pp_b = read_file(dir, "pp_b.i32", 4, n_pp);
  p.pp_v2 = read_file(dir, "pp_v2.f64", 8, n_pp);

  rtbte_options o;
  rtbte_default_options(&o);
  rtbte_ctx *ctx = NULL;
  if (rtbte_create(&p, 1, &o, &ctx) != RTBTE_OK) {
    fprintf(stderr, "rtbte_create: %s\n", rtbte_last_error(NULL));
    return 1;
  }
  const int64_t ny = rtbte_ny(ctx);
  double *y_h = read_file(dir, "y.f64", 8, ny);
  double *ydot_h = malloc((size_t)ny * sizeof(double));
  double *y_d = NULL, *ydot_d = NULL;
  if (!ydot_h || hipMalloc((void **)&y_d, (size_t)ny * sizeof(double)) != hipSuccess ||
      hipMalloc((void **)&ydot_d, (size_t)ny * sizeof(double)) != hipSuccess ||
      hipMemcpy(y_d, y_h, (size_t)ny * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    fprintf(stderr, "device buffers failed\n");
    return 1;
  }
  if (rtbte_rhs(ctx, y_d, ydot_d, RTBTE_PART_ALL, NULL) != RTBTE_OK) {
    fprintf(stderr, "rtbte_rhs: %s\n", rtbte_last_error(ctx));
    return 1;
  }
  if (hipMemcpy(ydot_h, ydot_d, (size_t)ny * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
    fprintf(stderr, "copy back failed\n");
    return 1;
  }
  snprintf(path, sizeof path, "%s/ydot.f64", dir);
  FILE *f = fopen(path, "wb");
  if (!f || fwrite(ydot_h, sizeof(double), (size_t)ny, f) != (size_t)ny) {
    fprintf(stderr, "cannot write %s\n", path);
    return 1;
  }
  fclose(f);
  int64_t counts[3];
  rtbte_counts(ctx, -1, counts);
  printf("%lld %lld %lld\n", (long long)counts[0], (long long)counts[1], (long long)counts[2]);
  if (argc == 3) {
    const double t_out = atof(argv[2]);
    const double zero = 0.0;
    double *t_d = NULL, *h_d = NULL;
    if (hipMalloc((void **)&t_d, sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&h_d, sizeof(double)) != hipSuccess ||
        hipMemcpy(t_d, &zero, sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h_d, &zero, sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
      fprintf(stderr, "device scalars failed\n");
      return 1;
    }
    if (rtbte_step_adaptive(ctx, y_d, t_d, h_d, t_out, 0, NULL) != RTBTE_OK) {
      fprintf(stderr, "rtbte_step_adaptive: %s\n", rtbte_last_error(ctx));
      return 1;
    }
    if (hipMemcpy(y_h, y_d, (size_t)ny * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
      fprintf(stderr, "copy back failed\n");
      return 1;
    }
    snprintf(path, sizeof path, "%s/y_out.f64", dir);
    FILE *g = fopen(path, "wb");
    if (!g || fwrite(y_h, sizeof(double), (size_t)ny, g) != (size_t)ny) {
      fprintf(stderr, "cannot write %s\n", path);
      return 1;
    }
    fclose(g);
    rtbte_stats st;
    if (rtbte_get_stats(ctx, 0, &st) != RTBTE_OK) {
      fprintf(stderr, "rtbte_get_stats: %s\n", rtbte_last_error(ctx));
      return 1;
    }
    printf("%lld %lld\n", (long long)st.n_accept, (long long)st.n_reject);
    (void)hipFree(t_d);
    (void)hipFree(h_d);
  }
  (void)hipFree(y_d);
  (void)hipFree(ydot_d);
  rtbte_destroy(ctx);
  return 0;
}
