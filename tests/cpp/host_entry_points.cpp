// Host-only entry points of the C ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer (built and run by tests/test_host_sanitizers.py;
// no device call is made): the planner over many shapes, variants and radix
// requests, the error paths, the twiddle generator, the tuning-table parser
// and the batched form's argument checks.  Exit status 0 when every call
// returned the status it should.
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <vector>

#include "pafc.h"

static int failures = 0;

static void expect(bool ok, const char* what, long long a, long long b) {
  if (!ok) {
    ++failures;
    std::fprintf(stderr, "FAIL %s (%lld, %lld)\n", what, a, b);
  }
}

static bool smooth(int64_t n) {
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

int main() {
  std::vector<char> buf(1 << 20);
  size_t need = 0;
  // 1-D: every length up to 3000 and a few large ones, every variant
  const pafc_variant vars[] = {PAFC_PERM_FREE, PAFC_EXPLICIT_PERM, PAFC_PERM_FREE_UNFUSED};
  for (int64_t n = 2; n <= 3000; ++n)
    for (pafc_variant v : vars)
      for (pafc_dtype dt : {PAFC_C128, PAFC_C64}) {
        const int64_t d[1] = {n};
        const pafc_status st = pafc_describe(1, d, nullptr, dt, v, buf.data(), buf.size(), &need);
        expect(st == PAFC_SUCCESS, "describe 1-D", n, (long long)v);
        expect(need > 2 && need <= buf.size() && std::strlen(buf.data()) + 1 == need,
               "describe length", n, (long long)need);
      }
  for (int64_t n : {65536LL, 78125LL, 1953125LL, 995329LL, 1000003LL, 7776000LL, 1LL << 22}) {
    const int64_t d[1] = {n};
    expect(pafc_describe(1, d, nullptr, PAFC_C128, PAFC_PERM_FREE, buf.data(), buf.size(),
                         &need) == PAFC_SUCCESS, "describe large", n, 0);
  }
  // truncated output: still NUL-terminated, `need` reports the full size
  {
    const int64_t d[1] = {4096};
    char small[16];
    expect(pafc_describe(1, d, nullptr, PAFC_C128, PAFC_PERM_FREE, small, sizeof(small), &need) ==
               PAFC_SUCCESS && small[15] == 0 && need > sizeof(small), "truncation", 0, 0);
  }
  // multi-D: smooth shapes accepted, a non-smooth axis rejected
  for (int64_t a : {2, 3, 12, 81, 100, 2187})
    for (int64_t b : {2, 9, 48, 125, 729, 4096})
      for (int64_t c : {0, 2, 20, 64}) {
        const int64_t d[3] = {a, b, c};
        const int nd = c ? 3 : 2;
        expect(pafc_describe(nd, d, nullptr, PAFC_C128, PAFC_PERM_FREE, buf.data(), buf.size(),
                             &need) == PAFC_SUCCESS, "describe multi-D", a * b, c);
      }
  {
    const int64_t d[2] = {7, 4};
    expect(pafc_describe(2, d, nullptr, PAFC_C128, PAFC_PERM_FREE, buf.data(), buf.size(),
                         &need) == PAFC_ERROR_UNSUPPORTED_SIZE, "non-smooth 2-D", 7, 4);
  }
  // uniform radix requests
  for (int r : {2, 3, 4, 5, 8})
    for (int64_t n : {16LL, 27LL, 64LL, 125LL, 243LL, 512LL, 3125LL, 4096LL}) {
      const int64_t d[1] = {n};
      const int rad[1] = {r};
      int64_t m = n;
      while (m % r == 0) m /= r;
      const pafc_status want = m == 1 ? PAFC_SUCCESS : PAFC_ERROR_UNSUPPORTED_SIZE;
      expect(pafc_describe(1, d, rad, PAFC_C128, PAFC_PERM_FREE, buf.data(), buf.size(),
                           &need) == want, "radix request", n, r);
    }
  // invalid arguments
  {
    const int64_t d[4] = {8, 8, 8, 8};
    expect(pafc_describe(0, d, nullptr, PAFC_C128, PAFC_PERM_FREE, buf.data(), buf.size(),
                         &need) == PAFC_ERROR_INVALID_VALUE, "ndim 0", 0, 0);
    expect(pafc_describe(4, d, nullptr, PAFC_C128, PAFC_PERM_FREE, buf.data(), buf.size(),
                         &need) == PAFC_ERROR_INVALID_VALUE, "ndim 4", 4, 0);
    const int64_t one[1] = {1};
    expect(pafc_describe(1, one, nullptr, PAFC_C128, PAFC_PERM_FREE, buf.data(), buf.size(),
                         &need) == PAFC_ERROR_INVALID_VALUE, "n = 1", 1, 0);
    expect(pafc_describe(1, d, nullptr, (pafc_dtype)7, PAFC_PERM_FREE, buf.data(), buf.size(),
                         &need) == PAFC_ERROR_INVALID_VALUE, "dtype", 7, 0);
    pafc_plan_t p = nullptr;
    expect(pafc_plan(nullptr, 1, d, nullptr, PAFC_C128, PAFC_PERM_FREE, nullptr) ==
               PAFC_ERROR_INVALID_VALUE, "plan NULL out", 0, 0);
    expect(pafc_plan(&p, 0, d, nullptr, PAFC_C128, PAFC_PERM_FREE, nullptr) ==
               PAFC_ERROR_INVALID_VALUE && p == nullptr, "plan ndim 0", 0, 0);
    expect(pafc_destroy(nullptr) == PAFC_SUCCESS, "destroy NULL", 0, 0);
  }
  // twiddles: the unit circle, conjugate symmetry
  for (int64_t n : {1LL, 3LL, 8LL, 27LL, 3125LL, 1953125LL, 1LL << 30})
    for (int64_t e = 0; e < 64; ++e) {
      double re = 0, im = 0, re2 = 0, im2 = 0;
      expect(pafc_twiddle(n, e * 7919 % n, &re, &im) == PAFC_SUCCESS, "twiddle", n, e);
      expect(pafc_twiddle(n, (n - e * 7919 % n) % n, &re2, &im2) == PAFC_SUCCESS, "twiddle", n, e);
      const double r2 = re * re + im * im;
      expect(r2 > 1 - 1e-15 && r2 < 1 + 1e-15 && re == re2 && im == -im2, "twiddle value", n, e);
    }
  expect(pafc_twiddle(0, 0, nullptr, nullptr) == PAFC_ERROR_INVALID_VALUE, "twiddle args", 0, 0);
  // tuning table parser
  expect(pafc_set_tuning("c128 65536 1024 0 0 0 0\nc64 4096 0 2 0 0 0 # note\n") == PAFC_SUCCESS,
         "tuning valid", 0, 0);
  for (const char* bad : {"garbage", "c128 x 1", "c99 64 0 0 0 0 0", "c128 64 0 0 0 9 0",
                          "c128 -5 0 0 0 0 0"})
    expect(pafc_set_tuning(bad) != PAFC_SUCCESS, "tuning invalid", 0, 0);
  expect(pafc_set_tuning(nullptr) == PAFC_SUCCESS, "tuning reset", 0, 0);
  // batched form: argument checks before any device call
  {
    pafc_batch_t b = nullptr;
    const int64_t sizes[3] = {64, 97, 64};
    const int fids[3] = {0, 1, 0};
    for (pafc_batch_form form : {PAFC_BATCH_PERSISTENT, PAFC_BATCH_LEVELS, PAFC_BATCH_CLASSES}) {
      expect(pafc_batch_plan(&b, 3, sizes, fids, 2, PAFC_C128, form, nullptr) ==
                 PAFC_ERROR_UNSUPPORTED_SIZE && b == nullptr, "batch non-smooth", form, 0);
      const int bad_fids[3] = {0, 0, 0};
      const int64_t sizes2[3] = {64, 128, 64};
      expect(pafc_batch_plan(&b, 3, sizes2, bad_fids, 1, PAFC_C128, form, nullptr) ==
                 PAFC_ERROR_INVALID_VALUE && b == nullptr, "batch filter sizes", form, 0);
      expect(pafc_batch_plan(&b, 0, sizes, fids, 1, PAFC_C128, form, nullptr) ==
                 PAFC_ERROR_INVALID_VALUE, "batch count", form, 0);
    }
    expect(pafc_batch_plan(&b, 3, sizes, fids, 2, PAFC_C128, (pafc_batch_form)7, nullptr) ==
               PAFC_ERROR_INVALID_VALUE && b == nullptr, "batch form", 0, 0);
  }
  for (int s = 0; s <= 6; ++s) expect(pafc_status_string((pafc_status)s) != nullptr, "status", s, 0);
  int smooth_count = 0;
  for (int64_t n = 2; n <= 3000; ++n) smooth_count += smooth(n);
  std::printf("host entry points: %d failures (%d smooth lengths, all 2..3000 planned)\n",
              failures, smooth_count);
  return failures == 0 ? 0 : 1;
}
