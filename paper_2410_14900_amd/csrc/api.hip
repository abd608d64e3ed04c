// Host side of the C ABI: validation, plan construction in float64, argument
// checking and dispatch to the kernel launchers.  Nothing here allocates or
// synchronises inside a stage call.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "dc_internal.h"

namespace dc {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

static dc_status fail(dc_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

static dc_status validate(const dc_grid* g, const dc_view* views, int32_t n) {
  std::string err;
  const dc_status st = validate_geometry(g, views, n, &err);
  if (st != DC_OK) set_error(err);
  return st;
}


// Derives the plan's tables for shape ks and uploads them (replacing any earlier
// tables of the plan): plan creation and knob changes.
static dc_status upload_tables(Plan* p, const dc_view* views, const KernelShape& ks);

dc_status set_shape(Plan* p, const KernelShape& ks) { return upload_tables(p, p->views.data(), ks); }

KernelShape shape_of(const dc_knobs& k) {
  KernelShape ks;
  ks.splat_kc = k.splat_angles;
  ks.interp_tx = k.interp_tile_u;
  ks.interp_kc = k.interp_angles;
  ks.bp_by = k.bp_block_y;
  ks.fp_ti = k.fp_tile_u;
  return ks;
}

dc_knobs knobs_of(const KernelShape& ks) {
  dc_knobs k{};
  k.splat_angles = ks.splat_kc;
  k.interp_tile_u = ks.interp_tx;
  k.interp_angles = ks.interp_kc;
  k.bp_block_y = ks.bp_by;
  k.fp_tile_u = ks.fp_ti;
  return k;
}

static dc_status build_plan(const dc_grid* g, const dc_view* views, int32_t n, const int32_t* first,
                            int32_t n_samples, Plan* p) {
  p->grid = *g;
  p->n_views = n;
  p->n_samples = n_samples;
  p->first.assign(first, first + n_samples + 1);
  KGrid& k = p->kg;
  k.nu = g->nu; k.nv = g->nv; k.n_theta = g->n_theta; k.n_s = g->n_s;
  k.nx = g->nx; k.ny = g->ny; k.nz = g->nz;
  k.du = (float)g->du; k.dv = (float)g->dv; k.ds = (float)g->ds;
  k.cu = 0.5f * (g->nu - 1); k.cv = 0.5f * (g->nv - 1);

  p->views.assign(views, views + n);
  const dc_status st = upload_tables(p, views, KernelShape());
  if (st != DC_OK) return st;
  hipError_t e;
  if ((e = hipMalloc((void**)&p->d_scratch, (n + n_samples) * sizeof(unsigned))) != hipSuccess ||
      (e = hipMalloc((void**)&p->d_masked, (size_t)n_samples * g->nx * g->ny *
                                               ((g->nz + kConeBrick - 1) / kConeBrick * kConeBrick) * sizeof(float))) !=
          hipSuccess)
    return fail(e == hipErrorOutOfMemory ? DC_ENOMEM : DC_EHIP, std::string("plan scratch: ") + hipGetErrorString(e));
  return DC_OK;
}

static dc_status upload_tables(Plan* p, const dc_view* views, const KernelShape& ks) {
  const dc_grid* g = &p->grid;
  const int n = p->n_views, n_samples = p->n_samples;
  HostPlan hp;
  std::string err;
  const dc_status st = plan_tables(g, views, n, p->first.data(), n_samples, ks, &hp, &err);
  if (st != DC_OK) return fail(st, err);
  // upload into new buffers; the plan keeps its old tables unless all succeed
  enum { kAng, kTrig, kView, kFrame, kProj, kRmax2, kChunks, kFirst, kForm, kN };
  void* fresh[kN] = {};
  const std::vector<int> forms(hp.cone_form.begin(), hp.cone_form.end());
  const void* src[kN] = {hp.ang.data(), hp.trig.data(), hp.vf.data(), hp.frame.data(),
                         hp.proj.data(), hp.rmax2.data(), hp.chunks.data(), p->first.data(), forms.data()};
  const size_t bytes[kN] = {hp.ang.size() * sizeof(double), hp.trig.size() * sizeof(float),
                            hp.vf.size() * sizeof(float), hp.frame.size() * sizeof(double),
                            hp.proj.size() * sizeof(double), hp.rmax2.size() * sizeof(float),
                            hp.chunks.size() * sizeof(int), p->first.size() * sizeof(int),
                            forms.size() * sizeof(int)};
  hipError_t e = hipSuccess;
  for (int i = 0; i < kN && e == hipSuccess; ++i) {
    e = hipMalloc(&fresh[i], bytes[i]);
    if (e == hipSuccess) e = hipMemcpy(fresh[i], src[i], bytes[i], hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    for (void* q : fresh)
      if (q) (void)hipFree(q);
    return fail(e == hipErrorOutOfMemory ? DC_ENOMEM : DC_EHIP, std::string("plan upload: ") + hipGetErrorString(e));
  }
  // the old tables may still be read by queued kernels: let the device drain first
  void* old[kN] = {p->d_ang, p->d_trig, p->d_view, p->d_frame, p->d_proj, p->d_rmax2, p->d_chunks, p->d_first,
                   p->d_form};
  bool any_old = false;
  for (void* q : old) any_old = any_old || q;
  if (any_old) {
    (void)hipDeviceSynchronize();
    for (void* q : old)
      if (q) (void)hipFree(q);
  }
  p->d_ang = (double*)fresh[kAng];
  p->d_trig = (float*)fresh[kTrig];
  p->d_view = (float*)fresh[kView];
  p->d_frame = (double*)fresh[kFrame];
  p->d_proj = (double*)fresh[kProj];
  p->d_rmax2 = (float*)fresh[kRmax2];
  p->d_chunks = (int4*)fresh[kChunks];
  p->d_first = (int*)fresh[kFirst];
  p->d_form = (int*)fresh[kForm];
  p->shape = ks;
  p->shape.splat_kc = hp.splat_kc;
  p->interp_wl = hp.interp_wl;
  p->splat_kc = hp.splat_kc;
  p->splat_max_terms = hp.splat_max_terms;
  p->splat_checked = hp.splat_checked;
  p->n_chunks = hp.n_chunks;
  p->cone_max_terms = hp.cone_max_terms;
  p->bp_stage = hp.bp_stage;
  p->bp_pitch = hp.bp_pitch;
  p->cone_form = hp.cone_form;
  p->splat_qmax = fixed_point_qmax(hp.splat_max_terms);
  p->cone_qmax = fixed_point_qmax(hp.cone_max_terms);
  return DC_OK;
}

static void free_plan(Plan* p) {
  void* ptrs[] = {p->d_ang,    p->d_trig,  p->d_view,    p->d_frame,  p->d_proj,   p->d_rmax2,
                  p->d_chunks, p->d_first, p->d_form,    p->d_scratch, p->d_masked};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete p;
}

void sample_span(const Plan& p, int v0, int nv, int* s_lo, int* s_hi) {
  // last sample whose first view is <= v
  auto sample_of = [&](int v) {
    int lo = 0, hi = p.n_samples - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (p.first[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
  };
  *s_lo = sample_of(v0);
  *s_hi = nv > 0 ? sample_of(v0 + nv - 1) : *s_lo;
}

// ---------------------------------------------------------- call checking
static dc_status check_call(const dc_plan plan, int32_t v0, int32_t nv) {
  if (!plan) return fail(DC_EINVAL, "null plan");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  if (v0 < 0 || nv < 0 || (int64_t)v0 + nv > p->n_views)
    return fail(DC_ESHAPE, "view range [" + std::to_string(v0) + ", " + std::to_string((int64_t)v0 + nv) +
                               ") outside [0, " + std::to_string(p->n_views) + ")");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return fail(DC_EINVAL, "current HIP device differs from the plan's device");
  return DC_OK;
}

static dc_status check_ptr(const void* q, const char* name, bool nullable = false) {
  if (!q) return nullable ? DC_OK : fail(DC_EINVAL, std::string("null pointer: ") + name);
  if (reinterpret_cast<uintptr_t>(q) % 16 != 0)
    return fail(DC_EALIGN, std::string("pointer not 16-byte aligned: ") + name);
  return DC_OK;
}

static dc_status check_dtype(dc_dtype t, const char* name) {
  if (t != DC_F32 && t != DC_BF16 && t != DC_F16) return fail(DC_EDTYPE, std::string("bad dtype for ") + name);
  return DC_OK;
}

static dc_status launched(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(DC_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return DC_OK;
}

#define DC_TRY(x)                  \
  do {                             \
    dc_status _st = (x);           \
    if (_st != DC_OK) return _st;  \
  } while (0)

}  // namespace dc

using namespace dc;

extern "C" {

const char* dc_last_error(void) { return g_last_error.c_str(); }

dc_status dc_validate(const dc_grid* grid, const dc_view* views, int32_t n_views) {
  return validate(grid, views, n_views);
}

static dc_status create(const dc_grid* grid, const dc_view* views, int32_t n_views, const int32_t* first,
                        int32_t n_samples, uint32_t flags, dc_plan* out) {
  if (!out) return fail(DC_EINVAL, "null output plan pointer");
  if (flags != 0) return fail(DC_EINVAL, "flags must be 0");
  DC_TRY(validate(grid, views, n_views));
  if (n_samples < 1) return fail(DC_ESHAPE, "n_samples must be >= 1");
  if (!first) return fail(DC_EINVAL, "null first_view");
  if (first[0] != 0 || first[n_samples] != n_views)
    return fail(DC_ESHAPE, "first_view must start at 0 and end at n_views");
  for (int s = 0; s < n_samples; ++s)
    if (first[s + 1] <= first[s])
      return fail(DC_ESHAPE, "sample " + std::to_string(s) + " has no views (first_view must increase)");
  const int bz = KernelShape().bp_bz;
  if ((long long)((grid->nz + bz - 1) / bz) * n_samples > 65535)
    return fail(DC_ENOTSUP, "too many samples for this volume depth (the backprojection grid holds "
                            "(nz / " + std::to_string(bz) + ") x samples <= 65535 blocks)");
  Plan* p = new Plan();
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return fail(DC_EHIP, "no HIP device");
  }
  dc_status st = build_plan(grid, views, n_views, first, n_samples, p);
  if (st != DC_OK) {
    free_plan(p);
    return st;
  }
  // set-up of the allocation-free entry point on this device (a failure here is
  // reported by that entry point, which repeats the lookup)
  unsigned* words = nullptr;
  (void)static_scratch(p->device, &words);
  *out = reinterpret_cast<dc_plan>(p);
  return DC_OK;
}

dc_status dc_plan_create(const dc_grid* grid, const dc_view* views, int32_t n_views, uint32_t flags,
                         dc_plan* out) {
  const int32_t first[2] = {0, n_views};
  return create(grid, views, n_views, first, 1, flags, out);
}

dc_status dc_plan_create_batched(const dc_grid* grid, const dc_view* views, int32_t n_views,
                                 const int32_t* first_view, int32_t n_samples, uint32_t flags, dc_plan* out) {
  return create(grid, views, n_views, first_view, n_samples, flags, out);
}

dc_status dc_plan_bounds(const dc_grid* grid, const dc_view* views, int32_t n_views, dc_bounds* out) {
  if (!out) return fail(DC_EINVAL, "null output bounds pointer");
  DC_TRY(validate(grid, views, n_views));
  HostPlan hp;
  std::string err;
  const int32_t first[2] = {0, n_views};
  const dc_status st = plan_tables(grid, views, n_views, first, 1, KernelShape(), &hp, &err);
  if (st != DC_OK) return fail(st, err);
  dc_bounds b{};
  b.splat_angles = hp.splat_kc;
  b.splat_max_terms = hp.splat_max_terms;
  b.splat_checked = hp.splat_checked;
  b.interp_window = hp.interp_wl;
  b.interp_local = hp.interp_wl > kInterpLocalAbove ? 1 : 0;
  b.cone_max_terms = hp.cone_max_terms;
  b.bp_stage = hp.bp_stage;
  b.bp_pitch = hp.bp_pitch;
  b.cone_form = hp.cone_form[0];
  b.splat_qmax = fixed_point_qmax(hp.splat_max_terms);
  b.cone_qmax = fixed_point_qmax(hp.cone_max_terms);
  const KernelShape ks;
  b.bp_block[0] = ks.bp_bx;
  b.bp_block[1] = ks.bp_by;
  b.bp_block[2] = ks.bp_bz;
  b.interp_tile[0] = ks.interp_tx;
  b.interp_tile[1] = ks.interp_ty;
  *out = b;
  return DC_OK;
}

dc_status dc_plan_get_knobs(dc_plan plan, dc_knobs* out) {
  if (!plan || !out) return fail(DC_EINVAL, "null argument");
  *out = knobs_of(reinterpret_cast<Plan*>(plan)->shape);
  return DC_OK;
}

dc_status dc_plan_set_knobs(dc_plan plan, const dc_knobs* knobs) {
  if (!plan || !knobs) return fail(DC_EINVAL, "null argument");
  Plan* p = reinterpret_cast<Plan*>(plan);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return fail(DC_EINVAL, "current HIP device differs from the plan's device");
  return set_shape(p, shape_of(*knobs));
}

dc_status dc_plan_autotune(dc_plan plan, uint32_t flags, hipStream_t stream, dc_knobs* chosen, double* ms,
                           int32_t* source) {
  if (!plan) return fail(DC_EINVAL, "null plan");
  if (flags != 0) return fail(DC_EINVAL, "flags must be 0");
  Plan* p = reinterpret_cast<Plan*>(plan);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return fail(DC_EINVAL, "current HIP device differs from the plan's device");
  return autotune(p, stream, chosen, ms, source);
}

dc_status dc_plan_destroy(dc_plan plan) {
  if (!plan) return fail(DC_EINVAL, "null plan");
  free_plan(reinterpret_cast<Plan*>(plan));
  return DC_OK;
}

int32_t dc_plan_n_views(dc_plan plan) { return plan ? reinterpret_cast<Plan*>(plan)->n_views : -1; }
int32_t dc_plan_n_samples(dc_plan plan) { return plan ? reinterpret_cast<Plan*>(plan)->n_samples : -1; }

dc_status dc_plan_grid(dc_plan plan, dc_grid* out) {
  if (!plan || !out) return fail(DC_EINVAL, "null argument");
  *out = reinterpret_cast<Plan*>(plan)->grid;
  return DC_OK;
}

dc_status dc_weight_radon(dc_plan plan, const float* g, void* R, dc_dtype tR, int32_t v0, int32_t nv,
                          hipStream_t stream) {
  DC_TRY(check_call(plan, v0, nv));
  DC_TRY(check_ptr(g, "g"));
  DC_TRY(check_ptr(R, "R"));
  DC_TRY(check_dtype(tR, "R"));
  if (nv == 0) return DC_OK;
  const Plan& p = *reinterpret_cast<Plan*>(plan);
  float scale = (float)(p.grid.du * p.grid.dv / p.grid.ds);
  return launched(launch_splat(p, g, DC_F32, true, scale, R, tR, v0, nv, stream), "dc_weight_radon");
}

dc_status dc_weight_radon_noalloc(dc_plan plan, const float* g, void* R, dc_dtype tR, int32_t v0, int32_t nv,
                                  hipStream_t stream) {
  DC_TRY(check_call(plan, v0, nv));
  DC_TRY(check_ptr(g, "g"));
  DC_TRY(check_ptr(R, "R"));
  DC_TRY(check_dtype(tR, "R"));
  if (nv > kNoAllocViews)
    return fail(DC_ESHAPE, "dc_weight_radon_noalloc takes at most " + std::to_string(kNoAllocViews) +
                               " views per call (its static scratch holds one word per view); got " +
                               std::to_string(nv));
  if (nv == 0) return DC_OK;
  const Plan& p = *reinterpret_cast<Plan*>(plan);
  unsigned* words = nullptr;
  const hipError_t e = static_scratch(p.device, &words);
  if (e != hipSuccess) return fail(DC_EHIP, std::string("static scratch address: ") + hipGetErrorString(e));
  float scale = (float)(p.grid.du * p.grid.dv / p.grid.ds);
  return launched(launch_splat(p, g, DC_F32, true, scale, R, tR, v0, nv, stream, words), "dc_weight_radon_noalloc");
}

dc_status dc_weight_radon_adjoint(dc_plan plan, const void* GR, dc_dtype tR, float* Gg, int32_t v0,
                                  int32_t nv, hipStream_t stream) {
  DC_TRY(check_call(plan, v0, nv));
  DC_TRY(check_ptr(GR, "GR"));
  DC_TRY(check_ptr(Gg, "Gg"));
  DC_TRY(check_dtype(tR, "GR"));
  if (nv == 0) return DC_OK;
  const Plan& p = *reinterpret_cast<Plan*>(plan);
  float scale = (float)(p.grid.du * p.grid.dv / p.grid.ds);
  return launched(launch_interp(p, GR, tR, true, scale, Gg, DC_F32, v0, nv, stream), "dc_weight_radon_adjoint");
}

dc_status dc_filter(dc_plan plan, const void* R, dc_dtype tR, const float* M, dc_wmode mode, void* H,
                    dc_dtype tH, int32_t v0, int32_t nv, hipStream_t stream) {
  DC_TRY(check_call(plan, v0, nv));
  DC_TRY(check_ptr(R, "R"));
  DC_TRY(check_ptr(M, "M"));
  DC_TRY(check_ptr(H, "H"));
  DC_TRY(check_dtype(tR, "R"));
  DC_TRY(check_dtype(tH, "H"));
  if (mode != DC_WEIGHT_ANALYTIC && mode != DC_WEIGHT_RAW) return fail(DC_EINVAL, "bad weight mode");
  if (nv == 0) return DC_OK;
  const Plan& p = *reinterpret_cast<Plan*>(plan);
  return launched(launch_filter(p, R, tR, M, mode == DC_WEIGHT_RAW, H, tH, v0, nv, stream), "dc_filter");
}

dc_status dc_filter_adjoint(dc_plan plan, const void* GH, dc_dtype tH, const void* R, dc_dtype tR,
                            const float* M, dc_wmode mode, float* GM, int32_t accumulate_GM, float* GR,
                            int32_t v0, int32_t nv, hipStream_t stream) {
  DC_TRY(check_call(plan, v0, nv));
  DC_TRY(check_ptr(GH, "GH"));
  DC_TRY(check_ptr(R, "R"));
  DC_TRY(check_ptr(M, "M"));
  DC_TRY(check_ptr(GM, "GM", true));
  DC_TRY(check_ptr(GR, "GR", true));
  DC_TRY(check_dtype(tH, "GH"));
  DC_TRY(check_dtype(tR, "R"));
  if (mode != DC_WEIGHT_ANALYTIC && mode != DC_WEIGHT_RAW) return fail(DC_EINVAL, "bad weight mode");
  if (nv == 0 || (!GM && !GR)) return DC_OK;
  const Plan& p = *reinterpret_cast<Plan*>(plan);
  return launched(launch_filter_adjoint(p, GH, tH, R, tR, M, mode == DC_WEIGHT_RAW, GM, accumulate_GM, GR,
                                        v0, nv, stream),
                  "dc_filter_adjoint");
}

dc_status dc_detector_bp(dc_plan plan, const void* H, dc_dtype tH, void* gF, dc_dtype tF, int32_t v0,
                         int32_t nv, hipStream_t stream) {
  DC_TRY(check_call(plan, v0, nv));
  DC_TRY(check_ptr(H, "H"));
  DC_TRY(check_ptr(gF, "gF"));
  DC_TRY(check_dtype(tH, "H"));
  DC_TRY(check_dtype(tF, "gF"));
  if (nv == 0) return DC_OK;
  const Plan& p = *reinterpret_cast<Plan*>(plan);
  float scale = (float)(M_PI / p.grid.n_theta);
  return launched(launch_interp(p, H, tH, false, scale, gF, tF, v0, nv, stream), "dc_detector_bp");
}

dc_status dc_detector_bp_adjoint(dc_plan plan, const void* GgF, dc_dtype tF, void* GH, dc_dtype tH,
                                 int32_t v0, int32_t nv, hipStream_t stream) {
  DC_TRY(check_call(plan, v0, nv));
  DC_TRY(check_ptr(GgF, "GgF"));
  DC_TRY(check_ptr(GH, "GH"));
  DC_TRY(check_dtype(tF, "GgF"));
  DC_TRY(check_dtype(tH, "GH"));
  if (nv == 0) return DC_OK;
  const Plan& p = *reinterpret_cast<Plan*>(plan);
  float scale = (float)(M_PI / p.grid.n_theta);
  return launched(launch_splat(p, GgF, tF, false, scale, GH, tH, v0, nv, stream), "dc_detector_bp_adjoint");
}

dc_status dc_cone_bp(dc_plan plan, const void* gF, dc_dtype tF, float* f, int32_t accumulate, int32_t relu,
                     int32_t v0, int32_t nv, hipStream_t stream) {
  DC_TRY(check_call(plan, v0, nv));
  DC_TRY(check_ptr(gF, "gF"));
  DC_TRY(check_ptr(f, "f"));
  DC_TRY(check_dtype(tF, "gF"));
  const Plan& p = *reinterpret_cast<Plan*>(plan);
  return launched(launch_cone_bp(p, gF, tF, f, accumulate, relu, v0, nv, stream), "dc_cone_bp");
}

dc_status dc_cone_bp_adjoint(dc_plan plan, const float* Gf, const float* f_relu, void* GgF, dc_dtype tF,
                             int32_t v0, int32_t nv, hipStream_t stream) {
  DC_TRY(check_call(plan, v0, nv));
  DC_TRY(check_ptr(Gf, "Gf"));
  DC_TRY(check_ptr(f_relu, "f_relu", true));
  DC_TRY(check_ptr(GgF, "GgF"));
  DC_TRY(check_dtype(tF, "GgF"));
  if (nv == 0) return DC_OK;
  const Plan& p = *reinterpret_cast<Plan*>(plan);
  return launched(launch_cone_fp(p, Gf, f_relu, GgF, tF, v0, nv, stream), "dc_cone_bp_adjoint");
}

static dc_status check_smooth(const Plan& p, double sigma, int32_t radius) {
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(DC_EINVAL, "sigma must be positive and finite");
  if (radius < 1 || radius > kSmoothMaxRadius)
    return fail(DC_EINVAL, "radius must be in [1, " + std::to_string(kSmoothMaxRadius) + "]");
  if (radius >= p.grid.n_theta || radius >= p.grid.n_s)
    return fail(DC_ESHAPE, "radius must be below n_theta and n_s (mirror padding)");
  if (smooth_mu_lds_bytes(p.grid.n_theta, radius) > kMaxLdsPerBlock)
    return fail(DC_ENOTSUP, "n_theta + 2 radius too large: the mu pass stages a column block of n_theta + 2 radius "
                            "rows in one workgroup's LDS (160 KiB)");
  return DC_OK;
}

dc_status dc_smooth_weights(dc_plan plan, const float* M, float* Ms, double sigma, int32_t radius, int32_t v0,
                            int32_t nv, hipStream_t stream) {
  DC_TRY(check_call(plan, v0, nv));
  DC_TRY(check_ptr(M, "M"));
  DC_TRY(check_ptr(Ms, "Ms"));
  const Plan& p = *reinterpret_cast<Plan*>(plan);
  DC_TRY(check_smooth(p, sigma, radius));
  if (nv == 0) return DC_OK;
  return launched(launch_smooth(p, M, Ms, sigma, radius, false, v0, nv, stream), "dc_smooth_weights");
}

dc_status dc_smooth_weights_adjoint(dc_plan plan, const float* GMs, float* GM, double sigma, int32_t radius,
                                    int32_t v0, int32_t nv, hipStream_t stream) {
  DC_TRY(check_call(plan, v0, nv));
  DC_TRY(check_ptr(GMs, "GMs"));
  DC_TRY(check_ptr(GM, "GM"));
  const Plan& p = *reinterpret_cast<Plan*>(plan);
  DC_TRY(check_smooth(p, sigma, radius));
  if (nv == 0) return DC_OK;
  return launched(launch_smooth(p, GMs, GM, sigma, radius, true, v0, nv, stream), "dc_smooth_weights_adjoint");
}

dc_status dc_project(dc_plan plan, const float* vol, float* g, int32_t v0, int32_t nv, hipStream_t stream) {
  DC_TRY(check_call(plan, v0, nv));
  DC_TRY(check_ptr(vol, "vol"));
  DC_TRY(check_ptr(g, "g"));
  if (nv == 0) return DC_OK;
  const Plan& p = *reinterpret_cast<Plan*>(plan);
  return launched(launch_project(p, vol, g, v0, nv, stream), "dc_project");
}

static dc_status check_segments(const dc_orbit_segment* segs, int32_t n_segs, int32_t fine, int n_views) {
  if (!segs) return fail(DC_EINVAL, "segs is NULL");
  if (n_segs < 1 || n_segs > crofton_max_segments())
    return fail(DC_EINVAL, "between 1 and " + std::to_string(crofton_max_segments()) + " orbit segments");
  if (fine < 1) return fail(DC_EINVAL, "fine must be at least 1");
  long long next = 0, samples = 0;
  for (int i = 0; i < n_segs; ++i) {
    const dc_orbit_segment& s = segs[i];
    const std::string id = "segment " + std::to_string(i) + ": ";
    if (s.kind < DC_SEG_CIRCLE || s.kind > DC_SEG_SINUSOID) return fail(DC_EINVAL, id + "unknown kind");
    if (s.start != next || s.count < 1) return fail(DC_EINVAL, id + "segments must cover the views in order");
    next += s.count;
    if (!std::isfinite(s.p0) || !std::isfinite(s.p1) || s.p1 == 0.0) return fail(DC_EINVAL, id + "bad parameters");
    if (s.closed != 0 && s.closed != 1) return fail(DC_EINVAL, id + "closed must be 0 or 1");
    if ((s.kind == DC_SEG_ARC || s.kind == DC_SEG_LINE) && s.closed) return fail(DC_EINVAL, id + "arcs and lines are open");
    if (s.kind == DC_SEG_SINUSOID && !s.closed) return fail(DC_EINVAL, id + "a sinusoid must be closed");
    if (!s.closed && s.count < 2) return fail(DC_EINVAL, id + "an open segment needs two views");
    if (s.closed && std::fabs(s.count * s.p1 - 2.0 * M_PI) > 1e-9)
      return fail(DC_EINVAL, id + "a closed segment must span one turn (count * p1 = 2 pi)");
    if (s.kind == DC_SEG_SINUSOID) {
      if (!std::isfinite(s.phi_max) || !std::isfinite(s.freq)) return fail(DC_EINVAL, id + "bad sinusoid");
      samples += (long long)fine * s.count;
    }
  }
  if (next != n_views) return fail(DC_EINVAL, "segments must cover all views of the plan");
  if (samples > (1ll << 24)) return fail(DC_ENOTSUP, "more than 2^24 sinusoid samples");
  return DC_OK;
}

size_t dc_crofton_workspace_bytes(const dc_orbit_segment* segs, int32_t n_segs, int32_t fine) {
  if (!segs || n_segs < 1 || n_segs > crofton_max_segments() || fine < 1) return 0;
  return crofton_workspace_bytes(segs, n_segs, fine);
}

dc_status dc_crofton_weights(dc_plan plan, const dc_orbit_segment* segs, int32_t n_segs, double sid, int32_t m_exp,
                             double taper, double c_floor, int32_t fine, float* M, int32_t v0, int32_t nv,
                             void* work, size_t work_bytes, hipStream_t stream) {
  DC_TRY(check_call(plan, v0, nv));
  const Plan& p = *reinterpret_cast<Plan*>(plan);
  if (p.n_samples != 1) return fail(DC_ENOTSUP, "the Crofton weight needs a plan of one scan");
  DC_TRY(check_segments(segs, n_segs, fine, p.n_views));
  if (!(sid > 0.0) || !std::isfinite(sid)) return fail(DC_EINVAL, "sid must be positive");
  if (m_exp < 1 || m_exp > 16) return fail(DC_EINVAL, "m_exp must be in [1, 16]");
  if (!(taper > 0.0 && taper <= 0.5)) return fail(DC_EINVAL, "taper must be in (0, 0.5]");
  if (!(c_floor > 0.0 && c_floor <= 1.0)) return fail(DC_EINVAL, "c_floor must be in (0, 1]");
  DC_TRY(check_ptr(M, "M"));
  DC_TRY(check_ptr(work, "work"));
  if (work_bytes < crofton_workspace_bytes(segs, n_segs, fine))
    return fail(DC_ESHAPE, "workspace smaller than dc_crofton_workspace_bytes()");
  if (nv == 0) return DC_OK;
  return launched(launch_crofton(p, segs, n_segs, sid, m_exp, taper, c_floor, fine, M, v0, nv, work, stream),
                  "dc_crofton_weights");
}

dc_status dc_poisson_noise(const float* p, float* out, int64_t* counts, size_t n, double photons, double mu,
                           uint64_t seed, uint64_t e0, hipStream_t stream) {
  if (!(photons > 0.0 && photons <= 1e12)) return fail(DC_EINVAL, "photons must be in (0, 1e12]");
  if (!(mu > 0.0) || !std::isfinite(mu)) return fail(DC_EINVAL, "mu must be positive");
  DC_TRY(check_ptr(p, "p"));
  DC_TRY(check_ptr(out, "out"));
  DC_TRY(check_ptr(counts, "counts", true));
  if (n == 0) return DC_OK;
  return launched(launch_poisson_noise(p, out, reinterpret_cast<long long*>(counts), n, photons, mu, seed, e0,
                                       stream),
                  "dc_poisson_noise");
}

dc_status dc_adam_step(float* M, const float* G, float* m, float* v, size_t n, const float* step, double lr,
                       double b1, double b2, double eps, double weight_decay, hipStream_t stream) {
  if (!(b1 >= 0.0 && b1 < 1.0 && b2 >= 0.0 && b2 < 1.0)) return fail(DC_EINVAL, "betas must lie in [0, 1)");
  if (!(eps > 0.0) || !std::isfinite(eps)) return fail(DC_EINVAL, "eps must be positive");
  if (!std::isfinite(lr)) return fail(DC_EINVAL, "lr must be finite");
  if (!(weight_decay >= 0.0) || !std::isfinite(weight_decay)) return fail(DC_EINVAL, "weight_decay must be >= 0");
  DC_TRY(check_ptr(M, "M"));
  DC_TRY(check_ptr(G, "G"));
  DC_TRY(check_ptr(m, "m"));
  DC_TRY(check_ptr(v, "v"));
  if (!step) return fail(DC_EINVAL, "null pointer: step");
  if (n == 0) return DC_OK;
  return launched(launch_adam(M, G, m, v, n, step, lr, b1, b2, eps, weight_decay, stream), "dc_adam_step");
}

size_t dc_ssim_workspace_bytes(int32_t nz, int32_t ny, int32_t nx) {
  if (nz < 11 || ny < 11 || nx < 11) return 0;
  return ssim_workspace_bytes(nz, ny, nx);
}

dc_status dc_ssim(const float* x, const float* y, int32_t nz, int32_t ny, int32_t nx, float data_range,
                  float* ssim, float* grad_x, void* work, size_t work_bytes, hipStream_t stream) {
  if (nz < 11 || ny < 11 || nx < 11) return fail(DC_ESHAPE, "every volume side must be at least 11 (the window)");
  if ((double)nz * ny * nx > 2147483647.0) return fail(DC_ESHAPE, "volume too large");
  if (!(data_range > 0.f) || !std::isfinite(data_range)) return fail(DC_EINVAL, "data_range must be positive");
  DC_TRY(check_ptr(x, "x"));
  DC_TRY(check_ptr(y, "y"));
  DC_TRY(check_ptr(ssim, "ssim"));
  DC_TRY(check_ptr(grad_x, "grad_x", true));
  DC_TRY(check_ptr(work, "work"));
  if (work_bytes < ssim_workspace_bytes(nz, ny, nx))
    return fail(DC_ESHAPE, "workspace smaller than dc_ssim_workspace_bytes()");
  return launched(launch_ssim(x, y, nz, ny, nx, data_range, ssim, grad_x, work, stream), "dc_ssim");
}

}  // extern "C"
