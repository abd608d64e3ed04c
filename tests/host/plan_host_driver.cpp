// Test driver for the host-only plan code: reads one geometry (int32 n_views,
// dc_grid, dc_view[n_views], raw little-endian) from the file named on the
// command line, runs the geometry check and the plan's float64 derivation, and
// prints the status and the bounds as one JSON line.  Built with host
// sanitizers by tests/test_plan_bounds.py, against the same source the library
// uses.
#include <cstdio>
#include <vector>

#include "plan_host.h"

int main(int argc, char** argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: %s geometry.bin\n", argv[0]);
    return 2;
  }
  std::FILE* fh = std::fopen(argv[1], "rb");
  if (!fh) return 2;
  int32_t n = 0;
  dc_grid g{};
  if (std::fread(&n, sizeof n, 1, fh) != 1 || std::fread(&g, sizeof g, 1, fh) != 1 || n < 0 || n > (1 << 20)) {
    std::fclose(fh);
    return 2;
  }
  std::vector<dc_view> views((size_t)n);
  if (n > 0 && std::fread(views.data(), sizeof(dc_view), (size_t)n, fh) != (size_t)n) {
    std::fclose(fh);
    return 2;
  }
  std::fclose(fh);
  std::string err;
  dc_status st = dc::validate_geometry(&g, views.data(), n, &err);
  dc::HostPlan hp;
  if (st == DC_OK) {
    const int first[2] = {0, n};
    st = dc::plan_tables(&g, views.data(), n, first, 1, dc::KernelShape(), &hp, &err);
  }
  if (st != DC_OK) {
    std::printf("{\"status\": %d}\n", (int)st);
    return 0;
  }
  double proj_sum = 0.0, ang_sum = 0.0;
  for (double x : hp.proj) proj_sum += x;
  for (double x : hp.ang) ang_sum += x;
  std::printf(
      "{\"status\": 0, \"splat_angles\": %d, \"splat_max_terms\": %d, \"splat_checked\": %d, "
      "\"interp_window\": %d, \"cone_max_terms\": %d, \"bp_stage\": %d, \"bp_pitch\": %d, \"cone_form\": %d, "
      "\"n_chunks\": %d, \"splat_qmax\": %.9g, \"cone_qmax\": %.9g, \"proj_sum\": %.17g, \"ang_sum\": %.17g}\n",
      hp.splat_kc, hp.splat_max_terms, hp.splat_checked, hp.interp_wl, hp.cone_max_terms, hp.bp_stage,
      hp.bp_pitch, (int)hp.cone_form[0], hp.n_chunks, (double)dc::fixed_point_qmax(hp.splat_max_terms),
      (double)dc::fixed_point_qmax(hp.cone_max_terms), proj_sum, ang_sum);
  return 0;
}
