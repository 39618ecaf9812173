// Host planning under AddressSanitizer and UndefinedBehaviorSanitizer: the planner of
// fm_plan_create (through fm_plan_inspect) over random problems of every boundary class,
// layout, precision, kind and Green's function, including invalid ones; fm_plan_create
// without a device (planning, then the failure and cleanup path); the host-only entry
// points with NULL and out-of-range arguments.  Exits non-zero on an unexpected status;
// the sanitizers abort on any memory or undefined-behaviour error.
#include <cstdio>
#include <random>

#include "../../include/fluxmi.h"

static int expect(bool ok, const char* what, int i) {
  if (!ok) std::fprintf(stderr, "unexpected: %s (case %d)\n", what, i);
  return ok ? 0 : 1;
}

int main() {
  std::mt19937 rng(12345);
  const int pairs[10][2] = {{2, 2}, {0, 0}, {1, 1}, {0, 1}, {1, 0}, {3, 3}, {0, 3}, {1, 3}, {3, 0}, {3, 1}};
  const int sizes[] = {1, 2, 3, 4, 5, 7, 8, 11, 12, 16, 22, 31, 32, 48, 64, 96, 100, 128, 243, 256, 512, 1000};
  int bad = 0, ok_count = 0;
  for (int i = 0; i < 4000; ++i) {
    int n[3], bc[3][2];
    double h[3];
    for (int a = 0; a < 3; ++a) {
      n[a] = sizes[rng() % (sizeof(sizes) / sizeof(int))];
      const int* p = pairs[rng() % 10];
      bc[a][0] = p[0];
      bc[a][1] = p[1];
      h[a] = 0.01 + 0.1 * (rng() % 1000) / 1000.0;
    }
    if (rng() % 50 == 0) bc[rng() % 3][rng() % 2] = 2;  // periodic on one face only
    if (rng() % 80 == 0) h[rng() % 3] = 0.0;
    if (rng() % 80 == 0) bc[rng() % 3][0] = 7;
    const int layout = rng() % 2, prec = rng() % 2, green = rng() % 9;
    const int kind = rng() % 5 == 0 ? 1 + rng() % 4 : 0;
    const int ncomp = kind ? 3 : 1 + rng() % 3;
    fm_plan_info info;
    const int rc = fm_plan_inspect(n, h, bc, layout, green, prec, kind, ncomp, &info);
    bad += expect(rc == FM_OK || (rc <= -2 && rc >= -4), fm_error_string(rc), i);
    if (rc == FM_OK) {
      ++ok_count;
      for (int p = 0; p < 5; ++p) bad += expect(info.tiles[p] >= 1 && info.lines_per_tile[p] >= 1, "tiling", i);
    }
    if (i % 40 == 0 && rc == FM_OK && (size_t)n[0] * n[1] * n[2] < (1u << 22)) {
      // the planner again through fm_plan_create; without a device it fails after planning
      fm_plan p = nullptr;
      const int rc2 = fm_plan_create(&p, n, h, bc, layout, green, prec, kind, ncomp, nullptr);
      if (rc2 == FM_OK) fm_plan_destroy(p);
      else bad += expect(p == nullptr, "plan left on failure", i);
    }
  }
  // fm_plan_create_vector over faces per component: mirror-symmetric sets (one axis
  // symmetric or semi-unbounded, or more, which the planner refuses) and broken ones;
  // without a device a plan that passes planning fails afterwards and is released
  int vec_planned = 0;
  for (int i = 0; i < 600; ++i) {
    int n[3], bcv[3][3][2];
    double h[3];
    for (int a = 0; a < 3; ++a) {
      n[a] = sizes[rng() % (sizeof(sizes) / sizeof(int))] % 200 + 2;
      h[a] = 0.01 + 0.1 * (rng() % 1000) / 1000.0;
      const int* pr = pairs[rng() % 10];
      for (int f = 0; f < 2; ++f)
        for (int q = 0; q < 3; ++q) {
          const int t = pr[f];
          // symmetric faces: the component along a swapped against the two others
          bcv[q][a][f] = (t <= 1 && q == a) ? 1 - t : t;
        }
    }
    if (rng() % 8 == 0) bcv[rng() % 3][rng() % 3][rng() % 2] = rng() % 4;  // may break the symmetry
    if (rng() % 40 == 0) bcv[rng() % 3][rng() % 3][rng() % 2] = 9;
    const int layout = rng() % 2, prec = rng() % 2, kind = 1 + rng() % 4;
    fm_plan p = nullptr;
    const int rc = fm_plan_create_vector(&p, n, h, bcv, layout, 0, prec, kind, nullptr);
    if (rc == FM_OK) fm_plan_destroy(p);
    else bad += expect(p == nullptr, "vector plan left on failure", i);
    bad += expect(rc == FM_OK || rc == FM_E_HIP || (rc <= -2 && rc >= -4), fm_error_string(rc), i);
    if (rc == FM_E_HIP) ++vec_planned;  // planning passed; the stubbed device refused
  }
  std::printf("vector plans through planning: %d of 600\n", vec_planned);
  // NULL and invalid arguments of the host-only entry points
  int n[3] = {8, 8, 8}, bc[3][2] = {{3, 3}, {3, 3}, {3, 3}};
  double h[3] = {0.1, 0.1, 0.1};
  fm_plan_info info;
  bad += expect(fm_plan_inspect(nullptr, h, bc, 0, 0, 0, 0, 1, &info) == FM_E_NULL, "inspect NULL n", 0);
  bad += expect(fm_plan_inspect(n, h, bc, 0, 0, 0, 0, 1, nullptr) == FM_E_NULL, "inspect NULL info", 0);
  bad += expect(fm_plan_inspect(n, h, bc, 5, 0, 0, 0, 1, &info) == FM_E_KIND, "inspect layout", 0);
  bad += expect(fm_plan_inspect(n, h, bc, 0, 0, 0, 0, 0, &info) == FM_E_KIND, "inspect ncomp", 0);
  bad += expect(fm_plan_create(nullptr, n, h, bc, 0, 0, 0, 0, 1, nullptr) == FM_E_NULL, "create NULL", 0);
  const int bv[3][3][2] = {{{3, 3}, {3, 3}, {1, 1}}, {{3, 3}, {3, 3}, {0, 0}}, {{3, 3}, {3, 3}, {0, 0}}};
  bad += expect(fm_plan_create_vector(nullptr, n, h, bv, 0, 0, 0, 1, nullptr) == FM_E_NULL, "vector NULL", 0);
  fm_plan pv = nullptr;
  bad += expect(fm_plan_create_vector(&pv, n, h, bv, 0, 0, 0, 0, nullptr) == FM_E_KIND, "vector Poisson", 0);
  bad += expect(fm_plan_destroy(nullptr) == FM_OK, "destroy NULL", 0);
  size_t bytes = 0;
  bad += expect(fm_plan_workspace_bytes(nullptr, &bytes) == FM_E_NULL, "workspace NULL", 0);
  bad += expect(fm_batched_workspace_bytes(0, nullptr, &bytes) != FM_OK, "batched count 0", 0);
  for (int e = -20; e <= 2; ++e) bad += expect(fm_error_string(e) != nullptr, "error string", e);
  std::printf("planned %d of 4000 problems, %d unexpected\n", ok_count, bad);
  return bad ? 1 : 0;
}
