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

static inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static inline void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

static dc_status validate(const dc_grid* g, const dc_view* views, int32_t n) {
  if (!g || !views) return fail(DC_EINVAL, "null grid or views");
  if (n < 1) return fail(DC_ESHAPE, "n_views must be >= 1");
  if (g->nu < 1 || g->nv < 1 || g->n_theta < 1 || g->n_s < 2 || g->nx < 1 || g->ny < 1 || g->nz < 1)
    return fail(DC_ESHAPE, "grid sizes must be positive (n_s >= 2)");
  const double lim = 2147483647.0;
  if ((double)g->nu * g->nv > lim / 4 || (double)g->n_theta * g->n_s > lim / 4 ||
      (double)g->nx * g->ny * g->nz > lim / 4)
    return fail(DC_ESHAPE, "per-view image, sinogram or volume too large for 32-bit indexing");
  if (g->n_s > 4096) return fail(DC_ESHAPE, "n_s above 4096 not supported (sinogram rows are staged in LDS)");
  if (g->nz > 1024) return fail(DC_ESHAPE, "nz above 1024 not supported");
  if (!(g->du > 0 && g->dv > 0 && g->ds > 0 && g->vx > 0 && g->vy > 0 && g->vz > 0))
    return fail(DC_EINVAL, "pitches and voxel sizes must be positive");
  const double hx = 0.5 * g->nx * g->vx, hy = 0.5 * g->ny * g->vy, hz = 0.5 * g->nz * g->vz;
  for (int v = 0; v < n; ++v) {
    const dc_view& w = views[v];
    double nx_ = std::sqrt(dot3(w.ex, w.ex)), ny_ = std::sqrt(dot3(w.ey, w.ey));
    if (std::fabs(nx_ - 1) > 1e-9 || std::fabs(ny_ - 1) > 1e-9 || std::fabs(dot3(w.ex, w.ey)) > 1e-9)
      return fail(DC_EINVAL, "view " + std::to_string(v) + ": detector axes not orthonormal");
    double lz[3], d[3];
    cross3(w.ex, w.ey, lz);
    for (int c = 0; c < 3; ++c) d[c] = w.src[c] - w.det_center[c];
    double D = dot3(d, lz);
    if (!(D > 0)) return fail(DC_EINVAL, "view " + std::to_string(v) + ": source not in front of the detector");
    double off = 0;
    for (int c = 0; c < 3; ++c) off += (d[c] - D * lz[c]) * (d[c] - D * lz[c]);
    if (std::sqrt(off) > 1e-6 * D)
      return fail(DC_EINVAL, "view " + std::to_string(v) + ": source not on the detector normal through its centre");
    for (int corner = 0; corner < 8; ++corner) {
      double p[3] = {g->ox + ((corner & 1) ? hx : -hx), g->oy + ((corner & 2) ? hy : -hy),
                     g->oz + ((corner & 4) ? hz : -hz)};
      double U = 0;
      for (int c = 0; c < 3; ++c) U += (w.src[c] - p[c]) * lz[c];
      if (!(U > 1e-6 * D))
        return fail(DC_EINVAL, "view " + std::to_string(v) + ": volume not entirely in front of the source");
    }
  }
  return DC_OK;
}


// Largest number of voxel centres the cone adjoint may add into one accumulator
// (one detector cell in one view); its fixed-point quantum is 2^30 / this of the
// largest term, so beyond it the adjoint would lose float32 accuracy.
static const int kMaxCellTerms = 1 << 18;

// Upper bound on the voxel centres whose projection in view w falls in one
// detector cell [i, i+1) x [j, j+1) of fractional indices.  Points of the cell's
// frustum are x = a + U (alpha l_x + beta l_y - l_z), U the depth, the cell
// spanning du/D in alpha and dv/D in beta.  Slice the centre lattice along an
// axis k over which x_k - a_k keeps one sign on the box.  Two frustum points x1,
// x2 in one slice differ by U1 (delta - (delta_k / d2_k) d2), d2 = (x2 - a)/U2,
// delta = d1 - d2 = dalpha l_x + dbeta l_y; along an in-slice axis b that is at
// most  U_max (du/D |l_x,b - t l_x,k| + dv/D |l_y,b - t l_y,k|),
// t = (x2_b - a_b)/(x2_k - a_k), whose extremes over the box (a linear-fractional
// function with a denominator of fixed sign) sit at its corners.  A slice thus
// holds at most (floor(E_b/v_b)+1)(floor(E_c/v_c)+1) centres and the box has
// n_k slices; the smallest such product over the admissible axes is the bound.
static double cell_terms_bound(const dc_grid* g, const dc_view& w, double D,
                               const double X0[3], double umax) {
  const int n[3] = {g->nx, g->ny, g->nz};
  const double vs[3] = {g->vx, g->vy, g->vz};
  double corner[8][3];
  for (int c = 0; c < 8; ++c)
    for (int k = 0; k < 3; ++k) corner[c][k] = X0[k] + ((c >> k) & 1) * (n[k] - 1) * vs[k] - w.src[k];
  double best = 1e300;
  for (int k = 0; k < 3; ++k) {
    bool pos = true, neg = true;
    for (int c = 0; c < 8; ++c) {
      pos = pos && corner[c][k] > 0.0;
      neg = neg && corner[c][k] < 0.0;
    }
    if (!pos && !neg) continue;   // the source lies within the box's extent along k
    double count = n[k];
    for (int b = 0; b < 3; ++b) {
      if (b == k) continue;
      double tmin = 1e300, tmax = -1e300;
      for (int c = 0; c < 8; ++c) {
        const double t = corner[c][b] / corner[c][k];
        tmin = std::min(tmin, t);
        tmax = std::max(tmax, t);
      }
      const double sx = std::max(std::fabs(w.ex[b] - tmin * w.ex[k]), std::fabs(w.ex[b] - tmax * w.ex[k]));
      const double sy = std::max(std::fabs(w.ey[b] - tmin * w.ey[k]), std::fabs(w.ey[b] - tmax * w.ey[k]));
      const double E = umax * (g->du / D * sx + g->dv / D * sy);
      count *= std::floor(E / vs[b] * (1.0 + 1e-9)) + 1.0;
    }
    best = std::min(best, count);
  }
  return best;
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

  const int K = g->n_theta;
  std::vector<double> ang(3 * K);
  std::vector<float> trig(2 * K);
  const double x0 = -0.5 * (g->nu - 1) * g->du, y0 = -0.5 * (g->nv - 1) * g->dv;
  int wl = 0;
  for (int kk = 0; kk < K; ++kk) {
    double mu = kk * M_PI / K, c = std::cos(mu), s = std::sin(mu);
    double A = g->du * c / g->ds, B = g->dv * s / g->ds;
    double C = (x0 * c + y0 * s) / g->ds + 0.5 * (g->n_s - 1);
    ang[3 * kk] = A; ang[3 * kk + 1] = B; ang[3 * kk + 2] = C;
    trig[2 * kk] = (float)c; trig[2 * kk + 1] = (float)s;
    int w = (int)std::ceil((interp_tile(0) - 1) * std::fabs(A) + (interp_tile(1) - 1) * std::fabs(B)) + 4;
    if (w > wl) wl = w;
  }
  p->interp_wl = wl;
  // the window rows of a chunk of 32 angles take 32 wl 8 bytes of LDS (<= 128 KiB)
  if (wl > 512) return fail(DC_ENOTSUP, "detector pitch too coarse for the s-bin width (ds << du)");

  // Radon work list: runs of angles whose pixels spread fastest along rows
  // (|A| >= |B|, lanes walk i) or along columns (lanes walk j), cut into chunks.
  // LDS holds kc rows of (n_s + 1) 64-bit accumulators, at most 80 KiB so that two
  // workgroups share a CU's 160 KiB (1381 bins, a 976^2 detector: 7 angles, 15-17% faster than
  // the 5 a 64 KiB budget allows)
  const int kc = std::max(1, std::min(8, 10240 / (g->n_s + 1)));
  p->splat_kc = kc;
  // bound on pixels sharing one bin on one angle, and whether every pixel's
  // bin index stays in [-1, n_s - 1] (then the splat needs no range checks)
  {
    int max_terms = 1;
    bool inside = true;
    for (int kk = 0; kk < K; ++kk) {
      const double A = std::fabs(ang[3 * kk]), B = std::fabs(ang[3 * kk + 1]);
      const double per_row = A > 0 ? std::floor(1.0 / A) + 1 : 1e30;
      const double per_col = B > 0 ? std::floor(1.0 / B) + 1 : 1e30;
      const double terms = std::min(per_row * g->nv, per_col * g->nu);
      max_terms = std::max(max_terms, (int)std::min(terms, (double)g->nu * g->nv));
      for (int c = 0; c < 4; ++c) {
        const double t = ang[3 * kk + 2] + ((c & 1) ? (g->nu - 1) * ang[3 * kk] : 0.0) +
                         ((c & 2) ? (g->nv - 1) * ang[3 * kk + 1] : 0.0);
        if (!(t >= -0.999 && t < g->n_s - 0.001)) inside = false;
      }
    }
    p->splat_max_terms = max_terms;
    p->splat_checked = inside ? 0 : 1;
  }
  std::vector<int> chunks;
  for (int kk = 0; kk < K;) {
    int colmajor = std::fabs(ang[3 * kk + 1]) > std::fabs(ang[3 * kk]) ? 1 : 0;
    int e = kk;
    while (e < K && e - kk < kc &&
           (std::fabs(ang[3 * e + 1]) > std::fabs(ang[3 * e]) ? 1 : 0) == colmajor) ++e;
    chunks.insert(chunks.end(), {kk, e - kk, colmajor, 0});
    kk = e;
  }
  p->n_chunks = (int)chunks.size() / 4;

  std::vector<float> vf(4 * n), rmax2(n);
  std::vector<double> frame(12 * n);
  for (int v = 0; v < n; ++v)
    for (int c = 0; c < 3; ++c) {
      frame[12 * v + c] = views[v].src[c];
      frame[12 * v + 3 + c] = views[v].det_center[c];
      frame[12 * v + 6 + c] = views[v].ex[c];
      frame[12 * v + 9 + c] = views[v].ey[c];
    }
  std::vector<double> proj(12 * n), zrel(n);
  double max_cell_terms = 0.0;
  const double X0[3] = {-0.5 * (g->nx - 1) * g->vx + g->ox, -0.5 * (g->ny - 1) * g->vy + g->oy,
                        -0.5 * (g->nz - 1) * g->vz + g->oz};
  const double vs[3] = {g->vx, g->vy, g->vz};
  const double four_pi2 = 4.0 * M_PI * M_PI;
  for (int v = 0; v < n; ++v) {
    const dc_view& w = views[v];
    double lz[3], d[3];
    cross3(w.ex, w.ey, lz);
    for (int c = 0; c < 3; ++c) d[c] = w.src[c] - w.det_center[c];
    double D = dot3(d, lz);
    vf[4 * v] = (float)D;
    vf[4 * v + 1] = (float)(dot3(w.tangent, w.ex) / (four_pi2 * D));
    vf[4 * v + 2] = (float)(dot3(w.tangent, w.ey) / (four_pi2 * D));
    vf[4 * v + 3] = (float)(dot3(w.tangent, lz) / (four_pi2 * D * D));
    double rel0[3];
    for (int c = 0; c < 3; ++c) rel0[c] = X0[c] - w.src[c];
    double* P = &proj[12 * v];
    for (int c = 0; c < 3; ++c) {
      double dn = -vs[c] * lz[c] / D;
      P[c] = dn;
      P[4 + c] = vs[c] * w.ex[c] / g->du + 0.5 * (g->nu - 1) * dn;
      P[8 + c] = vs[c] * w.ey[c] / g->dv + 0.5 * (g->nv - 1) * dn;
    }
    double dn0 = -dot3(rel0, lz) / D;
    P[3] = dn0;
    // depth range over the box of voxel centres (affine, extremes at corners)
    double umin = 1e300, umax = 0.0;
    for (int corner = 0; corner < 8; ++corner) {
      double den = dn0;
      for (int c = 0; c < 3; ++c) {
        const int nn = c == 0 ? g->nx : c == 1 ? g->ny : g->nz;
        if (corner & (1 << c)) den += P[c] * (nn - 1);
      }
      umin = std::min(umin, den * D);
      umax = std::max(umax, den * D);
    }
    rmax2[v] = (float)((D / umin) * (D / umin) * (1.0 + 1e-6));
    zrel[v] = std::fabs(P[2]) / (umin / D);   // largest relative change of den per voxel step in z
    max_cell_terms = std::max(max_cell_terms, cell_terms_bound(g, w, D, X0, umax));
    P[7] = dot3(rel0, w.ex) / g->du + 0.5 * (g->nu - 1) * dn0;
    P[11] = dot3(rel0, w.ey) / g->dv + 0.5 * (g->nv - 1) * dn0;
  }

  if (max_cell_terms > (double)kMaxCellTerms)
    return fail(DC_ENOTSUP, "up to " + std::to_string((long long)max_cell_terms) +
                                " voxel centres can project into one detector cell (limit " +
                                std::to_string(kMaxCellTerms) + "); the detector is too coarse for the voxel grid");
  p->cone_max_terms = (int)std::max(1.0, max_cell_terms);
  // largest backprojection block footprint (same box rule as the kernel) ->
  // how many pixels each of the backprojection's threads stages per view
  {
    const int B[3] = {cone_bp_block(0), cone_bp_block(1), cone_bp_block(2)};
    const int nb[3] = {(g->nx + B[0] - 1) / B[0], (g->ny + B[1] - 1) / B[1], (g->nz + B[2] - 1) / B[2]};
    double worst = 0;
    for (int v = 0; v < n; ++v) {
      const double* P = &proj[12 * v];
      for (int bz = 0; bz < nb[2]; ++bz)
        for (int by = 0; by < nb[1]; ++by)
          for (int bx = 0; bx < nb[0]; ++bx) {
            const int lo[3] = {bx * B[0], by * B[1], bz * B[2]};
            const int hi[3] = {std::min(g->nx, lo[0] + B[0]) - 1, std::min(g->ny, lo[1] + B[1]) - 1,
                               std::min(g->nz, lo[2] + B[2]) - 1};
            double imin = 1e300, imax = -1e300, jmin = 1e300, jmax = -1e300;
            for (int c = 0; c < 8; ++c) {
              const double x = (c & 1) ? hi[0] : lo[0], y = (c & 2) ? hi[1] : lo[1], z = (c & 4) ? hi[2] : lo[2];
              const double den = x * P[0] + y * P[1] + z * P[2] + P[3];
              const double iu = (x * P[4] + y * P[5] + z * P[6] + P[7]) / den;
              const double jv = (x * P[8] + y * P[9] + z * P[10] + P[11]) / den;
              imin = std::min(imin, iu); imax = std::max(imax, iu);
              jmin = std::min(jmin, jv); jmax = std::max(jmax, jv);
            }
            // kernel box: [floor(min)-1, floor(max)+2], plus slack for float rounding
            const double w = std::floor(imax) - std::floor(imin) + 5, h = std::floor(jmax) - std::floor(jmin) + 5;
            worst = std::max(worst, w * h);
          }
    }
    const int need = (int)std::ceil(worst / (double)cone_bp_threads());
    p->bp_stage = need <= 4 ? 4 : need <= 8 ? 8 : need <= 12 ? 12 : need <= 16 ? 16 : 0;
    // Form of the cone kernels, decided per sample (so a batched plan computes what
    // each scan's own plan does).  den = U/D and num_u free of z on every view: a
    // voxel column keeps one u and one weight per view, formed once per column.
    // Otherwise, if den changes by at most 2.5e-4 of itself per voxel step, one
    // Newton step from the previous voxel's reciprocal leaves a relative error of
    // that change squared (< 6.3e-8, float rounding) and replaces the reciprocal.
    p->cone_form.assign(p->first.size() - 1, kConeZinv);
    for (size_t smp = 0; smp + 1 < p->first.size(); ++smp) {
      bool zinv = true;
      double worst = 0.0;
      for (int v = p->first[smp]; v < p->first[smp + 1]; ++v) {
        zinv = zinv && proj[12 * v + 2] == 0.0 && proj[12 * v + 6] == 0.0;
        worst = std::max(worst, zrel[v]);
      }
      p->cone_form[smp] = zinv ? kConeZinv : worst <= 2.5e-4 ? kConeNewton : kConeGeneral;
    }
  }
  auto up = [&](void** dst, const void* src, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(dst, bytes);
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  };
  hipError_t e;
  if ((e = up((void**)&p->d_ang, ang.data(), ang.size() * sizeof(double))) != hipSuccess ||
      (e = up((void**)&p->d_trig, trig.data(), trig.size() * sizeof(float))) != hipSuccess ||
      (e = up((void**)&p->d_view, vf.data(), vf.size() * sizeof(float))) != hipSuccess ||
      (e = up((void**)&p->d_frame, frame.data(), frame.size() * sizeof(double))) != hipSuccess ||
      (e = up((void**)&p->d_proj, proj.data(), proj.size() * sizeof(double))) != hipSuccess ||
      (e = up((void**)&p->d_rmax2, rmax2.data(), rmax2.size() * sizeof(float))) != hipSuccess ||
      (e = up((void**)&p->d_chunks, chunks.data(), chunks.size() * sizeof(int))) != hipSuccess ||
      (e = up((void**)&p->d_first, p->first.data(), p->first.size() * sizeof(int))) != hipSuccess ||
      (e = hipMalloc((void**)&p->d_scratch, (n + n_samples) * sizeof(unsigned))) != hipSuccess ||
      (e = hipMalloc((void**)&p->d_masked, (size_t)n_samples * g->nx * g->ny * g->nz * sizeof(float))) !=
          hipSuccess)
    return fail(e == hipErrorOutOfMemory ? DC_ENOMEM : DC_EHIP,
                std::string("plan upload: ") + hipGetErrorString(e));
  return DC_OK;
}

static void free_plan(Plan* p) {
  void* ptrs[] = {p->d_ang,    p->d_trig,  p->d_view,    p->d_frame,  p->d_proj,
                  p->d_rmax2,  p->d_chunks, p->d_first, p->d_scratch, p->d_masked};
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
  if ((long long)((grid->nz + cone_bp_block(2) - 1) / cone_bp_block(2)) * n_samples > 65535)
    return fail(DC_ENOTSUP, "too many samples for this volume depth (the backprojection grid holds "
                            "(nz / " + std::to_string(cone_bp_block(2)) + ") x samples <= 65535 blocks)");
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
