// Host-only part of a plan: geometry validation and the float64 derivation of
// every table and bound the kernels rely on.  Plain C++ (no device code and no
// HIP runtime calls), so the same source is also built with host sanitizers.
#pragma once

#include <cmath>
#include <string>
#include <vector>

#include "dcfbp.h"

namespace dc {

// Work shapes of the kernels (the plan's knobs), whose bounds the plan derives:
//   splat_kc   angles per splat workgroup (sinogram rows held in LDS), 1..8; 0 picks
//              the most that fit 80 KiB of LDS (two workgroups per CU);
//   interp_tx  detector-BP pixel tile width, 32 or 64 (height interp_ty = 64);
//   interp_kc  detector-BP angles per chunk, 16, 32 or 64;
//   bp_by      cone-BP voxel block rows, 16 or 32 (block bp_bx x bp_by x bp_bz = 16 x . x 8);
//   fp_ti      cone-FP detector tile width, 16, 20 or 24 (height 64).
// The defaults are the values hand-tuned on the 256^3 / 512^2 training workload.
struct KernelShape {
  int splat_kc = 0;
  int interp_tx = 64, interp_ty = 64, interp_kc = 32;
  int bp_bx = 16, bp_by = 32, bp_bz = 8;
  int fp_ti = 20;
  int bp_threads() const { return bp_bx * bp_by; }
};
// Largest LDS one workgroup may hold on gfx950 (bytes), and the interp's largest angle chunk.
static constexpr int kLdsPerWorkgroup = 160 * 1024;
static constexpr int kInterpMaxKC = 64;

// DC_OK if the shape is one the kernels are built for (DC_EINVAL otherwise, message in *err).
dc_status check_shape(const KernelShape& ks, std::string* err);

enum ConeForm : char { kConeGeneral = 0, kConeQuadratic = 1, kConeZinv = 2 };

// Largest number of voxel centres the cone adjoint may add into one accumulator
// (one detector cell in one view); its fixed-point quantum is about 2^-31 times
// this of the largest term, so beyond it the adjoint would lose float32 accuracy.
static constexpr int kMaxCellTerms = 1 << 18;
// Widest detector-BP window (intervals of one angle's sinogram row staged in LDS).
static constexpr int kMaxInterpWindow = 512;

// Integer units given to the largest term of a fixed-point sum (the splat's a
// and b sums, the cone FP's four tap sums) when at most max_terms terms share
// one signed 32-bit accumulator half: max_terms terms of at most qmax + 1 units
// each (the term rounded to an integer, with a unit to spare for the float
// rounding of its scale) keep the half's magnitude at most 2^31 - 1, and every
// term stays below 2^21 units, where the kernels' float rounding trick (adding
// 1.5 2^23) is exact.  Computed on the host and passed to the kernels as a float
// (an integer below 2^21, exact), so bounds and kernels share one value.
inline float fixed_point_qmax(int max_terms) {
  const double q = std::floor(2147483647.0 / (double)std::max(max_terms, 1)) - 1.0;
  return q < 2097152.0 ? (float)q : 2097152.0f;
}

struct HostPlan {
  // per angle k: A_k = du cos mu/ds, B_k = dv sin mu/ds, C_k = fractional bin of pixel (0,0)
  std::vector<double> ang;       // [n_theta][3]
  std::vector<float> trig;       // [n_theta][2]  cos mu, sin mu
  // per view: D, t.l_x/(4 pi^2 D), t.l_y/(4 pi^2 D), t.l_z/(4 pi^2 D^2)
  std::vector<float> vf;         // [V][4]
  std::vector<double> frame;     // [V][12] source, detector centre, l_x, l_y
  std::vector<double> proj;      // [V][12] rows den, num_u, num_v over (ix, iy, iz, 1)
  std::vector<float> rmax2;      // [V] bound of (D/U)^2 over the voxel box
  std::vector<int> chunks;       // splat work list (k0, count, column_major, 0)
  std::vector<char> cone_form;   // per sample
  int n_chunks = 0;
  int splat_kc = 0;              // angles per splat workgroup
  int splat_max_terms = 0;       // bound on pixels sharing one (angle, bin)
  int splat_checked = 1;         // 1: some pixel may land outside bins [-1, n_s)
  int interp_wl = 0;             // detector-BP window length
  int cone_max_terms = 0;        // bound on voxel centres per detector cell in one view
  int bp_stage = 0;              // staged rows per cone-BP thread and view (0: direct taps)
  int bp_pitch = 0;              // pixels between staged rows: 64 or 128 (0: direct taps)
};

// Geometry check of dc_validate; on failure *err holds the message.
dc_status validate_geometry(const dc_grid* g, const dc_view* views, int n, std::string* err);

// Every table and bound of a plan over n views in n_samples scans (views of
// scan s are [first[s], first[s+1])), for kernels of shape `ks`.  The geometry
// must have passed validate_geometry.  DC_ENOTSUP (message in *err) when a
// bound exceeds what the kernels support.
dc_status plan_tables(const dc_grid* g, const dc_view* views, int n, const int* first, int n_samples,
                      const KernelShape& ks, HostPlan* out, std::string* err);

}  // namespace dc
