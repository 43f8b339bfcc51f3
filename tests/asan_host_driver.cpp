// Host-only driver for the AddressSanitizer build of the library: exercises
// validation, workspace sizing, flop counts and the launch-plan self-checks
// (forward for every precision, adjoint for FP64/FP32), the closed-shell and
// NAF sizing calls, and the error paths, without any GPU call.  Device
// pointers are placeholders that are never dereferenced.
#include <cstdint>
#include <cstdio>

#include "ltriples.h"

static int fails = 0;
static void expect(int got, int want, const char* what) {
  if (got != want) {
    std::printf("%s: got %d want %d (%s)\n", what, got, want, ltriples_last_error());
    ++fails;
  }
}

int main() {
  static double placeholder[4];
  const int32_t shapes[][5] = {{5, 4, 30, 31, 120}, {4, 0, 21, 22, 40}, {3, 1, 400, 401, 48},
                               {6, 5, 45, 47, 96},  {3, 3, 70, 67, 64}, {2, 2, 4, 4, 9}};
  for (const auto& sh : shapes) {
    ltriples_domain d{};
    d.noa = sh[0]; d.nob = sh[1]; d.nva = sh[2]; d.nvb = sh[3]; d.naux = sh[4];
    const double** fields[] = {&d.t1a, &d.t1b, &d.t2aa, &d.t2bb, &d.t2ab, &d.Boo_a, &d.Bov_a, &d.Bvv_a, &d.Boo_b,
                               &d.Bov_b, &d.Bvv_b, &d.eo_a, &d.ev_a, &d.eo_b, &d.ev_b, &d.fov_a, &d.fov_b};
    for (auto f : fields) *f = placeholder;
    for (int prec = 0; prec < 4; ++prec) {
      size_t ws = 0;
      expect(ltriples_validate(&d, prec, nullptr), LT_OK, "validate");
      expect(ltriples_workspace_size(&d, prec, nullptr, &ws), LT_OK, "workspace");
      expect(ltriples_plan_check(&d, prec, nullptr, 0), LT_OK, "forward plan");
      if (prec <= 1) {
        expect(ltriples_backward_workspace_size(&d, prec, nullptr, &ws), LT_OK, "backward workspace");
        expect(ltriples_plan_check(&d, prec, nullptr, 1), LT_OK, "backward plan");
      }
      ltriples_options o{};
      o.build_chunk_mib = 1;
      o.batch_items = 3;
      expect(ltriples_plan_check(&d, prec, &o, 0), LT_OK, "forward plan, small chunks");
    }
    double f = 0;
    int64_t n = 0;
    expect(ltriples_flops(&d, nullptr, &f, &n), LT_OK, "flops");
    // item lists, good and bad
    const int32_t good[] = {0, 0, 1, 2};
    const int32_t bad[] = {0, 2, 1, 0};
    ltriples_options o{};
    o.items = good;
    o.n_items = 1;
    if (d.noa >= 3) expect(ltriples_validate(&d, LT_FP64, &o), LT_OK, "good item");
    o.items = bad;
    expect(ltriples_validate(&d, LT_FP64, &o), LT_ESHAPE, "bad item");
  }
  // closed shell and NAF sizing
  ltriples_rhf_domain r{};
  r.no = 4; r.nv = 10; r.naux = 20;
  r.t1 = r.tau = r.Boo = r.Bov = r.Bvv = r.eo = r.ev = r.fov = placeholder;
  size_t ws = 0;
  double f = 0;
  int64_t n = 0;
  expect(ltriples_rhf_workspace_size(&r, LT_BF16X3, nullptr, &ws), LT_OK, "rhf workspace");
  expect(ltriples_backward_rhf_workspace_size(&r, LT_FP32, nullptr, &ws), LT_OK, "rhf backward workspace");
  expect(ltriples_rhf_flops(&r, &f, &n), LT_OK, "rhf flops");
  ltriples_naf_input ni{};
  ni.no_a = 3; ni.nv_a = 5; ni.no_b = 2; ni.nv_b = 6; ni.nx = 20;
  ni.Ja = ni.Jb = placeholder;
  expect(ltriples_naf_workspace_size(&ni, &ws), LT_OK, "naf workspace");
  // error paths
  expect(ltriples_validate(nullptr, LT_FP64, nullptr), LT_EINVAL, "null domain");
  expect(ltriples_rhf_workspace_size(nullptr, LT_FP64, nullptr, &ws), LT_EINVAL, "null rhf");
  ni.Ja = nullptr;
  expect(ltriples_naf_workspace_size(&ni, &ws), LT_EINVAL, "null J");
  std::printf("host checks done, %d failures\n", fails);
  return fails != 0;
}
