// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "dcfbp.h"
#include "plan_host.h"

namespace dc {

// ----------------------------------------------------------------- storage
// Conversions between float32 arithmetic and the storage types of dc_dtype.
struct bf16_t { uint16_t bits; };

__device__ __forceinline__ float to_f32(float x) { return x; }
__device__ __forceinline__ float to_f32(bf16_t x) { return __uint_as_float(uint32_t(x.bits) << 16); }
__device__ __forceinline__ float to_f32(_Float16 x) { return float(x); }

template <typename T> __device__ __forceinline__ T from_f32(float x);
template <> __device__ __forceinline__ float from_f32<float>(float x) { return x; }
template <> __device__ __forceinline__ _Float16 from_f32<_Float16>(float x) { return _Float16(x); }
template <> __device__ __forceinline__ bf16_t from_f32<bf16_t>(float x) {
  // round to nearest even; NaN stays NaN (quiet bit forced)
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return bf16_t{uint16_t((u >> 16) | 0x40u)};
  u += 0x7fffu + ((u >> 16) & 1u);
  return bf16_t{uint16_t(u >> 16)};
}

// Calls f with a value of the storage type selected at run time.
template <typename F>
static inline hipError_t by_dtype(dc_dtype t, F&& f) {
  switch (t) {
    case DC_F32: return f(float{});
    case DC_BF16: return f(bf16_t{});
    default: return f(_Float16{});
  }
}

// ------------------------------------------------------------ kernel args
// Scalar description of the sampling grids passed by value to every kernel.
struct KGrid {
  int nu, nv, n_theta, n_s, nx, ny, nz;
  float du, dv, ds;
  float cu, cv;          // (nu-1)/2, (nv-1)/2
};

// Plan: host copy of the geometry plus small device tables.

// z-segment length of the cone adjoint: its gather reads the gradient in bricks of
// this many consecutive slices (nz rounded up to a multiple of it, zero-padded)
static constexpr int kConeBrick = 16;

struct Plan {
  int device = 0;
  dc_grid grid{};
  int n_views = 0;
  KGrid kg{};
  // per angle k (float64): A_k = du cos mu/ds, B_k = dv sin mu/ds,
  // C_k = fractional bin index of pixel (0,0)      -> t = i A + j B + C
  double* d_ang = nullptr;       // [n_theta][3]
  float* d_trig = nullptr;       // [n_theta][2]  cos mu, sin mu
  // per view (float32): D, t.l_x/(4 pi^2 D), t.l_y/(4 pi^2 D), t.l_z/(4 pi^2 D^2)
  float* d_view = nullptr;       // [V][4]
  // per view (float64) frame for ray tracing: source, detector centre, l_x, l_y
  double* d_frame = nullptr;     // [V][12]
  // per view (float64) projective map of voxel indices: rows den, num_u, num_v,
  // each with coefficients of (ix, iy, iz, 1); i* = num_u/den, j* = num_v/den,
  // den = U/D, weight (D/U)^2 = 1/den^2
  double* d_proj = nullptr;      // [V][12]
  float* d_rmax2 = nullptr;      // [V] upper bound of (D/U)^2 over the volume
  int cone_max_terms = 0;        // max voxels sharing one (pixel cell) index in one view
  int bp_stage = 0;              // staged rows per thread and view in the backprojection (0: global taps)
  int bp_pitch = 0;              // pixels between the staged rows (64 or 128)
  // splat (Radon) work list: angle chunks that stay on one side of the diagonal
  int4* d_chunks = nullptr;      // (k0, count, column_major, 0)
  // samples (scans) of a batched plan: views of sample s are [first[s], first[s+1]);
  // per-view arrays hold all samples' views, volumes one block per sample
  int n_samples = 1;
  std::vector<int> first;        // host copy, [n_samples + 1]
  // per sample, the form of the cone kernels: kConeGeneral, kConeQuadratic (den varies so
  // slowly along z that 1/den is a quadratic in z over a segment) or kConeZinv
  // (no view's den or num_u has a z-term: the detector's v axis stays along z)
  std::vector<char> cone_form;
  int* d_first = nullptr;        // [n_samples + 1]
  int* d_form = nullptr;         // [n_samples] cone_form on the device, for launches over mixed forms
  // plan-owned scratch: [0, V) per-view max |input| of the splat, [V, V + S) per-sample
  // max |Gf| of the cone adjoint (float bits, reduced with integer atomicMax).  Calls
  // on one plan must therefore be ordered on one stream.
  unsigned* d_scratch = nullptr; // [V + S]
  // volume-sized scratch for dc_cone_bp_adjoint: Gf (times [f > 0] with a ReLU
  // mask) rewritten once in z-bricks of kConeBrick voxels, zero-padded, which the
  // gather reads as contiguous 64-byte segments
  float* d_masked = nullptr;     // [S][ceil(nz/16)][ny][nx][16]
  int n_chunks = 0;
  int splat_kc = 0;              // max angles per chunk
  int splat_max_terms = 0;       // max pixels that share one (angle, bin)
  int splat_checked = 1;         // 0 when every pixel lands on bins [-1, n_s) for all angles
  int interp_wl = 0;             // LDS window length for the interpolating kernels
                                 // (above kInterpLocalAbove: the fixed-point position tap form)
  // fixed-point scales: a sum of the splat (cone FP) holds terms of at most qmax
  // units, qmax = fixed_point_qmax(splat_max_terms (cone_max_terms))
  float splat_qmax = 0.f, cone_qmax = 0.f;
  // the kernels' work shapes (knobs) the tables were derived for
  KernelShape shape;
  // host copy of the views, to re-derive the tables for another shape
  std::vector<dc_view> views;
};



void set_error(const std::string& msg);

// Re-derives and uploads the plan's tables for another kernel shape (api.hip);
// synchronises the device before freeing the old tables.
dc_status set_shape(Plan* p, const KernelShape& ks);
KernelShape shape_of(const dc_knobs& k);
dc_knobs knobs_of(const KernelShape& ks);
// dc_plan_autotune's search (autotune.hip)
dc_status autotune(Plan* p, hipStream_t s, dc_knobs* chosen, double* ms, int32_t* source);

static constexpr int kInterpLocalAbove = 160;

// samples whose views meet [v0, v0+nv): s_lo..s_hi; for an empty range the
// sample holding view v0 (the last one when v0 = V)
void sample_span(const Plan& p, int v0, int nv, int* s_lo, int* s_hi);

// Gaussian weight smoothing (smooth.hip): normalised taps w[|t|], t = -r..r
static constexpr int kSmoothMaxRadius = 255;
struct GaussTaps {
  float w[kSmoothMaxRadius + 1];
};
GaussTaps gauss_taps(double sigma, int r);
// LDS of the smoothing's mu pass (taps and a column block of n_theta + 2r rows);
// a workgroup may hold up to kMaxLdsPerBlock bytes on gfx950
size_t smooth_mu_lds_bytes(int n_theta, int r);
static constexpr size_t kMaxLdsPerBlock = 160 * 1024;
hipError_t launch_smooth(const Plan& p, const float* in, float* out, double sigma, int r, bool adjoint, int v0,
                         int nv, hipStream_t s);

// Siddon cone-beam projector (project.hip)
hipError_t launch_project(const Plan& p, const float* vol, float* g, int v0, int nv, hipStream_t s);

// smooth Crofton weight of eq. 9 (crofton.hip); segments already validated
int crofton_max_segments();
size_t crofton_workspace_bytes(const dc_orbit_segment* segs, int n_segs, int fine);
hipError_t launch_crofton(const Plan& p, const dc_orbit_segment* segs, int n_segs, double sid, int m_exp,
                          double taper, double c_floor, int fine, float* M, int v0, int nv, void* work,
                          hipStream_t s);

// Poisson noise with the Philox4x64-10 generator (noise.hip)
hipError_t launch_poisson_noise(const float* p, float* out, long long* counts, size_t n, double photons, double mu,
                                unsigned long long seed, unsigned long long e0, hipStream_t s);

// fused Adam / AdamW step (adam.hip)
hipError_t launch_adam(float* M, const float* G, float* m, float* v, size_t n, const float* step, double lr,
                       double b1, double b2, double eps, double wd, hipStream_t s);

// 3D SSIM and its gradient (ssim.hip)
size_t ssim_workspace_bytes(int nz, int ny, int nx);
hipError_t launch_ssim(const float* x, const float* y, int nz, int ny, int nx, float L, float* ssim, float* grad,
                       void* work, hipStream_t s);

// scratch helpers (radon2d.hip)
hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t s);

// launchers (return hipSuccess or the launch error)
// vmax_words: nv zeroed-then-reduced words for the per-view fixed-point scales
// (nullptr: the plan's scratch)
hipError_t launch_splat(const Plan& p, const void* img, dc_dtype t_in, bool wcos, float scale,
                        void* out, dc_dtype t_out, int v0, int nv, hipStream_t s, unsigned* vmax_words = nullptr);
// The allocation-free splat's static scratch (radon2d.hip): kNoAllocViews words per
// GPU; *out = its address on `device`, which must be current (looked up once per device).
static constexpr int kNoAllocViews = 65536;
static constexpr int kMaxDevices = 64;
hipError_t static_scratch(int device, unsigned** out);
hipError_t launch_interp(const Plan& p, const void* rows, dc_dtype t_in, bool wcos, float scale,
                         void* out, dc_dtype t_out, int v0, int nv, hipStream_t s);
hipError_t launch_filter(const Plan& p, const void* R, dc_dtype tR, const float* M, int raw,
                         void* H, dc_dtype tH, int v0, int nv, hipStream_t s);
hipError_t launch_filter_adjoint(const Plan& p, const void* GH, dc_dtype tH, const void* R,
                                 dc_dtype tR, const float* M, int raw, float* GM, int acc,
                                 float* GR, int v0, int nv, hipStream_t s);
hipError_t launch_cone_bp(const Plan& p, const void* gF, dc_dtype tF, float* f, int acc, int relu,
                          int v0, int nv, hipStream_t s);
hipError_t launch_cone_fp(const Plan& p, const float* Gf, const float* f_relu, void* GgF,
                          dc_dtype tF, int v0, int nv, hipStream_t s);

}  // namespace dc
