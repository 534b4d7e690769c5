/* The oracle's C routines under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built and run by tests/test_host_sanitizers.py,
 * serial: no OpenMP): the standard FFT route against the direct sum on small
 * 1-D, 2-D and 3-D shapes with several radix sequences, sampled direct sums,
 * and the digit-reversal permutation.  Exit status 0 when all agree. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_conv_direct(int ndim, const int64_t *dims, const double *x, const double *h, double *y);
int orc_conv_direct_at(int ndim, const int64_t *dims, const double *x, const double *h,
                       int64_t nidx, const int64_t *idx, double *out);
int orc_conv_fft(int ndim, const int64_t *dims, const int *rho_flat, const int *rho_len,
                 const double *x, const double *h, double *y);
int orc_perm_index(int64_t n, int t, const int *rho, int64_t *perm);

static int failures = 0;

static double rel(const double *a, const double *b, int64_t n2) {
  double num = 0, den = 0;
  for (int64_t i = 0; i < n2; ++i) {
    num += (a[i] - b[i]) * (a[i] - b[i]);
    den += b[i] * b[i];
  }
  return sqrt(num / den);
}

static void check(int ndim, const int64_t *dims, const int *rho, const int *len) {
  int64_t N = 1;
  for (int a = 0; a < ndim; ++a) N *= dims[a];
  double *x = malloc((size_t)N * 2 * sizeof(double)), *h = malloc((size_t)N * 2 * sizeof(double));
  double *y1 = malloc((size_t)N * 2 * sizeof(double)), *y2 = malloc((size_t)N * 2 * sizeof(double));
  uint64_t s = 88172645463325252ull;
  for (int64_t i = 0; i < 2 * N; ++i) {
    s ^= s << 13; s ^= s >> 7; s ^= s << 17;
    x[i] = (double)(s >> 11) / 9007199254740992.0 - 0.5;
    s ^= s << 13; s ^= s >> 7; s ^= s << 17;
    h[i] = (double)(s >> 11) / 9007199254740992.0 - 0.5;
  }
  if (orc_conv_direct(ndim, dims, x, h, y1) != 0 || orc_conv_fft(ndim, dims, rho, len, x, h, y2) != 0) {
    ++failures;
    fprintf(stderr, "FAIL status N=%lld\n", (long long)N);
  } else if (rel(y2, y1, 2 * N) > 1e-13) {
    ++failures;
    fprintf(stderr, "FAIL fft vs direct N=%lld: %g\n", (long long)N, rel(y2, y1, 2 * N));
  }
  int64_t idx[3] = {0, N / 2, N - 1};
  double at[6];
  if (orc_conv_direct_at(ndim, dims, x, h, 3, idx, at) != 0) ++failures;
  for (int k = 0; k < 3; ++k)
    if (at[2 * k] != y1[2 * idx[k]] || at[2 * k + 1] != y1[2 * idx[k] + 1]) {
      ++failures;
      fprintf(stderr, "FAIL direct_at N=%lld k=%d\n", (long long)N, k);
    }
  free(x); free(h); free(y1); free(y2);
}

int main(void) {
  { int64_t d[1] = {60}; int r[4] = {2, 2, 3, 5}, l[1] = {4}; check(1, d, r, l); }
  { int64_t d[1] = {60}; int r[3] = {5, 4, 3}, l[1] = {3}; check(1, d, r, l); }
  { int64_t d[1] = {64}; int r[2] = {8, 8}, l[1] = {2}; check(1, d, r, l); }
  { int64_t d[1] = {2}; int r[1] = {2}, l[1] = {1}; check(1, d, r, l); }
  { int64_t d[2] = {8, 9}; int r[4] = {2, 4, 3, 3}, l[2] = {2, 2}; check(2, d, r, l); }
  { int64_t d[3] = {4, 5, 6}; int r[4] = {4, 5, 2, 3}, l[3] = {1, 1, 2}; check(3, d, r, l); }
  /* perm_index: a permutation of 0..n-1 */
  {
    int rho[4] = {2, 3, 4, 5};
    int64_t perm[120];
    int seen[120] = {0};
    if (orc_perm_index(120, 4, rho, perm) != 0) ++failures;
    for (int i = 0; i < 120; ++i) {
      if (perm[i] < 0 || perm[i] >= 120 || seen[perm[i]]++) {
        ++failures;
        fprintf(stderr, "FAIL perm_index %d\n", i);
        break;
      }
    }
  }
  printf("oracle under sanitizers: %d failures\n", failures);
  return failures == 0 ? 0 : 1;
}
