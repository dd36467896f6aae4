/*
 * Sanitizer driver of the FP64 oracle (TEST INFRASTRUCTURE): built together
 * with shape_oracle.c under AddressSanitizer and UndefinedBehaviorSanitizer by
 * the CPU test suite, it runs every entry point that allocates or indexes
 * (single-pair estimate, fixed and adaptive screens with and without seeded
 * budgets, antithetic sampling, the series, the grid, the alignment gradient
 * and both Adam drivers, alignment starts, features, the network's loss and
 * gradient) on small deterministic molecules, and the parameter checks of the
 * screen.  Prints one line per call; exits non-zero on an unexpected return
 * code (the sanitizers abort on their own findings).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int or_estimate(int, const float*, const float*, uint32_t, int, const float*, const float*,
                uint32_t, int64_t, int64_t, uint64_t, int, double*);
int or_screen(int, const float*, const float*, uint32_t, int32_t, const int32_t*, const float*,
              const float*, const uint32_t*, const int32_t*, int32_t, int, int64_t, int64_t,
              int64_t, double, uint64_t, int, const int32_t*, int, double*);
double or_incexc(int, const float*, const float*, int, const float*, const float*);
int or_grid_integrals(int, const float*, const float*, int, const float*, const float*, double,
                      double, int, double*);
int or_align_grad(int, const float*, const float*, uint32_t, int, const float*, const float*,
                  uint32_t, int64_t, uint64_t, int32_t, const double*, double*, double*,
                  double*);
int or_align_adam(int, const float*, const float*, uint32_t, int, const float*, const float*,
                  uint32_t, int64_t, uint64_t, int32_t, const double*, int32_t, double, double*,
                  double*);
int or_fo_align_adam(int, const float*, const float*, int, const float*, const float*, int32_t,
                     const double*, int32_t, double, double*, double*);
int or_fo_starts(int, const float*, const float*, int, const float*, const float*, uint32_t,
                 int32_t, uint64_t, double*);
int or_features(int32_t, const int32_t*, const float*, const float*, double*);
int64_t or_mlp_nparams(int, const int32_t*);
int or_mlp_loss_grad(int, const int32_t*, const double*, int32_t, const double*, const double*,
                     const double*, double*, double*);

/* a zig-zag chain of n atoms, 1.5 A bonds, widths near those of C/N/O */
static void chain(int n, float shift, float* xyz, float* alpha) {
  for (int i = 0; i < n; ++i) {
    xyz[3 * i + 0] = 1.25f * (float)i + shift;
    xyz[3 * i + 1] = (i & 1) ? 0.8f : -0.1f * (float)(i % 3);
    xyz[3 * i + 2] = 0.3f * (float)((i * 7) % 5) - 0.6f;
    alpha[i] = 0.80f + 0.05f * (float)(i % 4);
  }
}

static int failures = 0;

static void expect(const char* what, int rc, int want) {
  printf("%-34s rc %d\n", what, rc);
  if (rc != want) {
    fprintf(stderr, "%s: return code %d, expected %d\n", what, rc, want);
    ++failures;
  }
}

int main(void) {
  enum { NQ = 9, NL = 5 };
  float xq[3 * NQ], aq[NQ];
  chain(NQ, 0.0f, xq, aq);
  /* library: molecules of 3, 7, 1, 12, 5 atoms in CSR order */
  const int32_t sizes[NL] = {3, 7, 1, 12, 5};
  int32_t off[NL + 1] = {0};
  for (int m = 0; m < NL; ++m) off[m + 1] = off[m] + sizes[m];
  const int natoms = off[NL];
  float* lx = (float*)malloc(sizeof(float) * 3 * natoms);
  float* la = (float*)malloc(sizeof(float) * natoms);
  for (int m = 0; m < NL; ++m) chain(sizes[m], 0.4f * (float)m, lx + 3 * off[m], la + off[m]);
  uint32_t ids[NL] = {11, 12, 13, 14, 15};

  double r20[20];
  expect("estimate iid", or_estimate(NQ, xq, aq, 1, 7, lx + 3 * off[1], la + off[1], 2, 1000,
                                     777, 5, 0, r20), 0);
  expect("estimate antithetic", or_estimate(NQ, xq, aq, 1, 7, lx + 3 * off[1], la + off[1], 2,
                                            1000, 778, 5, 1, r20), 0);

  const int32_t pairs[7] = {0, 4, 2, -1, 3, 5, 1};
  const int32_t budgets[7] = {0, 1000, 512, 0, 4096, 0, 9999};
  double* out6 = (double*)malloc(sizeof(double) * 6 * 7);
  expect("screen fixed", or_screen(NQ, xq, aq, 1, NL, off, lx, la, ids, pairs, 7, 0, 256, 0, 0,
                                   0.0, 3, 2, NULL, 0, out6), 0);
  expect("screen adaptive", or_screen(NQ, xq, aq, 1, NL, off, lx, la, ids, NULL, NL, 1, 0, 512,
                                      4096, 0.01, 3, 2, NULL, 0, out6), 0);
  expect("screen adaptive seeded", or_screen(NQ, xq, aq, 1, NL, off, lx, la, NULL, pairs, 7, 1,
                                             0, 512, 4096, 0.02, 3, 2, budgets, 0, out6), 0);
  expect("screen adaptive antithetic", or_screen(NQ, xq, aq, 1, NL, off, lx, la, ids, pairs, 7,
                                                 1, 0, 512, 2048, 0.02, 3, 1, NULL, 1, out6), 0);
  /* parameters the rounds cannot follow are refused before any allocation */
  expect("screen cap not whole rounds", or_screen(NQ, xq, aq, 1, NL, off, lx, la, ids, NULL,
                                                  NL, 1, 0, 512, 1000, 0.01, 3, 1, NULL, 0,
                                                  out6), -2);
  expect("screen odd round size", or_screen(NQ, xq, aq, 1, NL, off, lx, la, ids, NULL, NL, 1, 0,
                                            1, 4, 0.01, 3, 1, NULL, 0, out6), -2);

  double s = or_incexc(5, lx + 3 * off[4], la + off[4], 3, lx, la);
  printf("%-34s %.6f\n", "incexc", s);
  double g8[8];
  expect("grid", or_grid_integrals(3, lx, la, 5, lx + 3 * off[4], la + off[4], 0.3, 4.0, 2,
                                   g8), 0);

  double pose[2 * 7] = {1, 0, 0, 0, 0.2, -0.1, 0.3, 0.8, 0.2, -0.3, 0.1, -0.4, 0.5, 0.0};
  double T[2], G[14], self2[2], pose_out[14];
  expect("align grad", or_align_grad(NQ, xq, aq, 1, 12, lx + 3 * off[3], la + off[3], 14, 256,
                                     9, 2, pose, T, G, self2), 0);
  expect("align adam", or_align_adam(NQ, xq, aq, 1, 12, lx + 3 * off[3], la + off[3], 14, 256, 9,
                                     2, pose, 4, 0.05, pose_out, T), 0);
  expect("fo align adam", or_fo_align_adam(NQ, xq, aq, 12, lx + 3 * off[3], la + off[3], 2,
                                           pose, 4, 0.05, pose_out, T), 0);
  double starts[8 * 7];
  expect("fo starts", or_fo_starts(NQ, xq, aq, 7, lx + 3 * off[1], la + off[1], 3, 3, 5,
                                   starts), 0);

  double* feat = (double*)malloc(sizeof(double) * 24 * NL);
  expect("features", or_features(NL, off, lx, la, feat), 0);

  const int32_t width[4] = {6, 5, 4, 2};
  const int64_t np = or_mlp_nparams(3, width);
  double* prm = (double*)malloc(sizeof(double) * np);
  double* grad = (double*)malloc(sizeof(double) * np);
  for (int64_t i = 0; i < np; ++i) prm[i] = 0.1 * sin((double)i);
  double x[3 * 6], tgt[3 * 2], lw[2] = {1.0, 0.5}, loss;
  for (int i = 0; i < 18; ++i) x[i] = cos(0.3 * i);
  for (int i = 0; i < 6; ++i) tgt[i] = 0.1 * i;
  expect("mlp loss grad", or_mlp_loss_grad(3, width, prm, 3, x, tgt, lw, &loss, grad), 0);

  free(lx); free(la); free(out6); free(feat); free(prm); free(grad);
  if (failures) return 1;
  printf("sanitize driver ok\n");
  return 0;
}
