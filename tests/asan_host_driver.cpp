// Host-only driver for the sanitizer build of the library: exercises
// validation, workspace sizing, flop counts and the launch-plan self-checks
// (forward for every precision, adjoint for FP64/FP32/BF16X3) on small and full-size
// domains, the rejection of domains too large for any device, the
// closed-shell and NAF sizing calls, and the error paths, without any GPU
// call.  Device pointers are placeholders that are never dereferenced.
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

static ltriples_domain fake_domain(const int32_t (&sh)[5], const double* p) {
  ltriples_domain d{};
  d.noa = sh[0]; d.nob = sh[1]; d.nva = sh[2]; d.nvb = sh[3]; d.naux = sh[4];
  const double** fields[] = {&d.t1a, &d.t1b, &d.t2aa, &d.t2bb, &d.t2ab, &d.Boo_a, &d.Bov_a, &d.Bvv_a, &d.Boo_b,
                             &d.Bov_b, &d.Bvv_b, &d.eo_a, &d.ev_a, &d.eo_b, &d.ev_b, &d.fov_a, &d.fov_b};
  for (auto f : fields) *f = p;
  return d;
}

int main() {
  static double placeholder[4];
  const int32_t shapes[][5] = {{5, 4, 30, 31, 120}, {4, 0, 21, 22, 40}, {3, 1, 400, 401, 48},
                               {6, 5, 45, 47, 96},  {3, 3, 70, 67, 64}, {2, 2, 4, 4, 9}};
  for (const auto& sh : shapes) {
    ltriples_domain d = fake_domain(sh, placeholder);
    for (int prec = 0; prec < 4; ++prec) {
      size_t ws = 0;
      expect(ltriples_validate(&d, prec, nullptr), LT_OK, "validate");
      expect(ltriples_workspace_size(&d, prec, nullptr, &ws), LT_OK, "workspace");
      expect(ltriples_plan_check(&d, prec, nullptr, 0), LT_OK, "forward plan");
      if (prec <= 2) {
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
  // full-size shapes (the gradient, LNO-sized and largest domains): sizing,
  // flop counts and the forward plan, with byte offsets beyond 2^31
  const int32_t big[][5] = {{20, 18, 160, 162, 640}, {40, 38, 300, 302, 1200}, {60, 58, 500, 502, 2000}};
  for (const auto& sh : big) {
    ltriples_domain d = fake_domain(sh, placeholder);
    for (int prec = 0; prec < 3; ++prec) {
      size_t ws = 0;
      expect(ltriples_workspace_size(&d, prec, nullptr, &ws), LT_OK, "full-size workspace");
      if (ws < ((size_t)1 << 31)) expect(0, 1, "full-size workspace beyond 2 GiB");
      expect(ltriples_plan_check(&d, prec, nullptr, 0), LT_OK, "full-size forward plan");
    }
    size_t ws = 0;
    expect(ltriples_backward_workspace_size(&d, LT_FP32, nullptr, &ws), LT_OK, "full-size backward workspace");
    double f = 0;
    int64_t n = 0;
    expect(ltriples_flops(&d, nullptr, &f, &n), LT_OK, "full-size flops");
  }
  // domains no device can hold are rejected before any size is derived from
  // them: inputs over 1 TiB, and dimensions whose products would overflow
  const int32_t huge[][5] = {{40, 38, 20000, 20000, 1200}, {2000000000, 2000000000, 46340, 46340, 2000000000},
                             {4096, 4096, 46340, 46340, 1 << 24}, {3, 3, 30, 30, 2000000000}};
  for (const auto& sh : huge) {
    ltriples_domain d = fake_domain(sh, placeholder);
    size_t ws = 0;
    expect(ltriples_validate(&d, LT_FP32, nullptr), LT_ESHAPE, "oversized domain");
    expect(ltriples_workspace_size(&d, LT_FP32, nullptr, &ws), LT_ESHAPE, "oversized domain workspace");
  }
  {
    ltriples_rhf_domain r{};
    r.no = 2000000000; r.nv = 46340; r.naux = 2000000000;
    r.t1 = r.tau = r.Boo = r.Bov = r.Bvv = r.eo = r.ev = r.fov = placeholder;
    size_t ws = 0;
    expect(ltriples_rhf_workspace_size(&r, LT_FP32, nullptr, &ws), LT_ESHAPE, "oversized closed-shell domain");
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
  // option fields: forced tiles 0..8 per output layout, check_finite 0/1,
  // deterministic accepted with any value; the batched call checks them too
  {
    const int32_t sh[5] = {5, 4, 30, 31, 120};
    ltriples_domain d = fake_domain(sh, placeholder);
    ltriples_options o{};
    o.tile_override[0] = 8; o.tile_override[1] = 1; o.tile_override[2] = 0;
    o.deterministic = 7;
    o.check_finite = 1;
    expect(ltriples_validate(&d, LT_BF16X3, &o), LT_OK, "forced tiles in range");
    expect(ltriples_plan_check(&d, LT_FP64, &o, 0), LT_OK, "plan with forced tiles");
    o.tile_override[2] = 9;
    expect(ltriples_validate(&d, LT_FP32, &o), LT_EINVAL, "forced tile out of range");
    expect(ltriples_workspace_size_batched(&d, 1, LT_FP32, &o, &ws), LT_EINVAL, "batched forced tile out of range");
    o.tile_override[2] = -1;
    expect(ltriples_validate(&d, LT_FP32, &o), LT_EINVAL, "negative forced tile");
    o.tile_override[2] = 0;
    o.check_finite = 2;
    expect(ltriples_validate(&d, LT_FP32, &o), LT_EINVAL, "check_finite not 0/1");
  }
  // launch groups of the batched call: every budget packs 20 domains (more
  // than one group's 16) into regions that the sizing accounts for
  {
    ltriples_domain ds[20];
    for (int k = 0; k < 20; ++k) {
      const int32_t sh[5] = {3 + k % 5, 2 + k % 4, 20 + 7 * k, 19 + 5 * k, 40 + k};
      ds[k] = fake_domain(sh, placeholder);
    }
    size_t plain = 0;
    expect(ltriples_workspace_size_batched(ds, 20, LT_BF16X3, nullptr, &plain), LT_OK, "batched, no groups");
    const size_t budgets[] = {1, size_t(64) << 20, size_t(1) << 50};
    for (size_t b : budgets) {
      ltriples_options o{};
      o.group_budget = b;
      for (int prec = 0; prec < 4; ++prec) {
        size_t w = 0;
        expect(ltriples_workspace_size_batched(ds, 20, prec, &o, &w), LT_OK, "batched with groups");
      }
      size_t w = 0;
      expect(ltriples_workspace_size_batched(ds, 20, LT_BF16X3, &o, &w), LT_OK, "batched with groups");
      if (w < plain) {
        std::printf("group budget %zu: workspace %zu below the ungrouped %zu\n", b, w, plain);
        ++fails;
      }
    }
  }
  // central-orbital share sizing, both spins, every precision, small and LNO-sized
  {
    const double pts[3] = {0.2, 0.7, 1.9}, wts[3] = {0.3, 0.4, 0.6};
    const int32_t cs[][5] = {{5, 4, 30, 31, 120}, {3, 1, 17, 18, 30}, {40, 38, 300, 302, 1200}};
    for (const auto& sh : cs) {
      ltriples_domain d = fake_domain(sh, placeholder);
      for (int spin = 0; spin < 2; ++spin)
        for (int prec = 0; prec < 4; ++prec) {
          ltriples_central c{spin, placeholder, 3, pts, wts};
          expect(ltriples_central_workspace_size(&d, &c, prec, nullptr, &ws), LT_OK, "central workspace");
        }
    }
    ltriples_domain d = fake_domain(cs[0], placeholder);
    ltriples_central c{0, placeholder, 0, pts, wts};
    expect(ltriples_central_workspace_size(&d, &c, LT_FP64, nullptr, &ws), LT_EINVAL, "central nq = 0");
  }
  // debug W dump: argument and item checks (all before any device work)
  {
    const int32_t sh[5] = {5, 4, 30, 31, 120};
    ltriples_domain d = fake_domain(sh, placeholder);
    const int32_t good[4] = {1, 0, 1, 3}, bad[4] = {0, 2, 1, 3};
    double* wp = (double*)placeholder;
    expect(ltriples_debug_w(&d, LT_FP64, nullptr, wp, wp, nullptr, 0, nullptr), LT_EINVAL, "debug_w null item");
    expect(ltriples_debug_w(&d, LT_FP64, good, nullptr, wp, nullptr, 0, nullptr), LT_EINVAL, "debug_w null w");
    expect(ltriples_debug_w(&d, LT_FP64, bad, wp, wp, nullptr, 0, nullptr), LT_ESHAPE, "debug_w bad item");
  }
  // error paths
  expect(ltriples_validate(nullptr, LT_FP64, nullptr), LT_EINVAL, "null domain");
  expect(ltriples_rhf_workspace_size(nullptr, LT_FP64, nullptr, &ws), LT_EINVAL, "null rhf");
  ni.Ja = nullptr;
  expect(ltriples_naf_workspace_size(&ni, &ws), LT_EINVAL, "null J");
  std::printf("host checks done, %d failures\n", fails);
  return fails != 0;
}
