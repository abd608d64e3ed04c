// Host-only plan construction: validation and the float64 derivation of the
// kernels' tables and bounds (see plan_host.h).  No device code, no HIP calls.
#include "plan_host.h"

#include <algorithm>
#include <cmath>

namespace dc {

static inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static inline void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

static dc_status fail(std::string* err, dc_status st, const std::string& msg) {
  if (err) *err = msg;
  return st;
}

dc_status validate_geometry(const dc_grid* g, const dc_view* views, int n, std::string* err) {
  if (!g || !views) return fail(err, DC_EINVAL, "null grid or views");
  if (n < 1) return fail(err, DC_ESHAPE, "n_views must be >= 1");
  if (g->nu < 1 || g->nv < 1 || g->n_theta < 1 || g->n_s < 2 || g->nx < 1 || g->ny < 1 || g->nz < 1)
    return fail(err, DC_ESHAPE, "grid sizes must be positive (n_s >= 2)");
  const double lim = 2147483647.0;
  if ((double)g->nu * g->nv > lim / 4 || (double)g->n_theta * g->n_s > lim / 4 ||
      (double)g->nx * g->ny * g->nz > lim / 4)
    return fail(err, DC_ESHAPE, "per-view image, sinogram or volume too large for 32-bit indexing");
  if (g->n_s > 4096) return fail(err, DC_ESHAPE, "n_s above 4096 not supported (sinogram rows are staged in LDS)");
  if (g->nz > 1024) return fail(err, DC_ESHAPE, "nz above 1024 not supported");
  if (!(g->du > 0 && g->dv > 0 && g->ds > 0 && g->vx > 0 && g->vy > 0 && g->vz > 0))
    return fail(err, DC_EINVAL, "pitches and voxel sizes must be positive");
  const double hx = 0.5 * g->nx * g->vx, hy = 0.5 * g->ny * g->vy, hz = 0.5 * g->nz * g->vz;
  for (int v = 0; v < n; ++v) {
    const dc_view& w = views[v];
    double nx_ = std::sqrt(dot3(w.ex, w.ex)), ny_ = std::sqrt(dot3(w.ey, w.ey));
    if (!(std::fabs(nx_ - 1) <= 1e-9 && std::fabs(ny_ - 1) <= 1e-9 && std::fabs(dot3(w.ex, w.ey)) <= 1e-9))
      return fail(err, DC_EINVAL, "view " + std::to_string(v) + ": detector axes not orthonormal");
    double lz[3], d[3];
    cross3(w.ex, w.ey, lz);
    for (int c = 0; c < 3; ++c) d[c] = w.src[c] - w.det_center[c];
    double D = dot3(d, lz);
    if (!(D > 0)) return fail(err, DC_EINVAL, "view " + std::to_string(v) + ": source not in front of the detector");
    double off = 0;
    for (int c = 0; c < 3; ++c) off += (d[c] - D * lz[c]) * (d[c] - D * lz[c]);
    if (!(std::sqrt(off) <= 1e-6 * D))
      return fail(err, DC_EINVAL,
                  "view " + std::to_string(v) + ": source not on the detector normal through its centre");
    for (int corner = 0; corner < 8; ++corner) {
      double p[3] = {g->ox + ((corner & 1) ? hx : -hx), g->oy + ((corner & 2) ? hy : -hy),
                     g->oz + ((corner & 4) ? hz : -hz)};
      double U = 0;
      for (int c = 0; c < 3; ++c) U += (w.src[c] - p[c]) * lz[c];
      if (!(U > 1e-6 * D))
        return fail(err, DC_EINVAL, "view " + std::to_string(v) + ": volume not entirely in front of the source");
    }
  }
  return DC_OK;
}

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
static double cell_terms_bound(const dc_grid* g, const dc_view& w, double D, const double X0[3], double umax) {
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

dc_status check_shape(const KernelShape& ks, std::string* err) {
  if (ks.splat_kc < 0 || ks.splat_kc > 8) return fail(err, DC_EINVAL, "splat angles per workgroup must be 0..8");
  if (ks.interp_tx != 32 && ks.interp_tx != 64) return fail(err, DC_EINVAL, "detector-BP tile width must be 32 or 64");
  if (ks.interp_ty != 64) return fail(err, DC_EINVAL, "detector-BP tile height must be 64");
  if (ks.interp_kc != 16 && ks.interp_kc != 32 && ks.interp_kc != 64)
    return fail(err, DC_EINVAL, "detector-BP angles per chunk must be 16, 32 or 64");
  if (ks.bp_bx != 16 || ks.bp_bz != 8 || (ks.bp_by != 16 && ks.bp_by != 32))
    return fail(err, DC_EINVAL, "cone-BP block must be 16 x 16 x 8 or 16 x 32 x 8");
  if (ks.fp_ti != 16 && ks.fp_ti != 20 && ks.fp_ti != 24) return fail(err, DC_EINVAL, "cone-FP tile width must be 16, 20 or 24");
  return DC_OK;
}

dc_status plan_tables(const dc_grid* g, const dc_view* views, int n, const int* first, int n_samples,
                      const KernelShape& ks, HostPlan* p, std::string* err) {
  {
    const dc_status st = check_shape(ks, err);
    if (st != DC_OK) return st;
  }
  const int K = g->n_theta;
  p->ang.assign(3 * K, 0.0);
  p->trig.assign(2 * K, 0.f);
  const double x0 = -0.5 * (g->nu - 1) * g->du, y0 = -0.5 * (g->nv - 1) * g->dv;
  int wl = 0;
  for (int kk = 0; kk < K; ++kk) {
    double mu = kk * M_PI / K, c = std::cos(mu), s = std::sin(mu);
    double A = g->du * c / g->ds, B = g->dv * s / g->ds;
    double C = (x0 * c + y0 * s) / g->ds + 0.5 * (g->n_s - 1);
    p->ang[3 * kk] = A;
    p->ang[3 * kk + 1] = B;
    p->ang[3 * kk + 2] = C;
    p->trig[2 * kk] = (float)c;
    p->trig[2 * kk + 1] = (float)s;
    // a tile's pixels span (tx-1)|A| + (ty-1)|B| bins; the window holds those
    // intervals, one below the first and margins for rounding
    int w = (int)std::ceil((ks.interp_tx - 1) * std::fabs(A) + (ks.interp_ty - 1) * std::fabs(B)) + 4;
    if (w > wl) wl = w;
  }
  p->interp_wl = wl;
  if (wl > kMaxInterpWindow)
    return fail(err, DC_ENOTSUP, "detector pitch too coarse for the s-bin width (ds << du): detector-BP window of " +
                                     std::to_string(wl) + " intervals (limit " + std::to_string(kMaxInterpWindow) + ")");
  // the window rows of one angle chunk, 8 bytes per interval, plus the kernel's
  // own per-angle tables (under 4 KiB), in one workgroup's LDS
  if ((long long)ks.interp_kc * wl * 8 + 4096 > kLdsPerWorkgroup)
    return fail(err, DC_ENOTSUP, "detector-BP window of " + std::to_string(wl) + " intervals x " +
                                     std::to_string(ks.interp_kc) + " angles exceeds a workgroup's LDS");

  // Radon work list: runs of angles whose pixels spread fastest along rows
  // (|A| >= |B|, lanes walk i) or along columns (lanes walk j), cut into chunks.
  // LDS holds kc rows of (n_s + 1) 64-bit accumulators, at most 80 KiB so that two
  // workgroups share a CU's 160 KiB (1381 bins, a 976^2 detector: 7 angles, 15-17%
  // faster than the 5 a 64 KiB budget allows)
  int kc = ks.splat_kc > 0 ? ks.splat_kc : std::max(1, std::min(8, 10240 / (g->n_s + 1)));
  if ((long long)kc * (g->n_s + 1) * 8 + 1024 > kLdsPerWorkgroup)
    return fail(err, DC_ENOTSUP, std::to_string(kc) + " sinogram rows of " + std::to_string(g->n_s) +
                                     " bins per splat workgroup exceed its LDS");
  p->splat_kc = kc;
  // bound on pixels sharing one bin on one angle, and whether every pixel's
  // bin index stays in [-1, n_s - 1] (then the splat needs no range checks)
  {
    int max_terms = 1;
    bool inside = true;
    for (int kk = 0; kk < K; ++kk) {
      const double A = std::fabs(p->ang[3 * kk]), B = std::fabs(p->ang[3 * kk + 1]);
      const double per_row = A > 0 ? std::floor(1.0 / A) + 1 : 1e30;
      const double per_col = B > 0 ? std::floor(1.0 / B) + 1 : 1e30;
      const double terms = std::min(per_row * g->nv, per_col * g->nu);
      max_terms = std::max(max_terms, (int)std::min(terms, (double)g->nu * g->nv));
      for (int c = 0; c < 4; ++c) {
        const double t = p->ang[3 * kk + 2] + ((c & 1) ? (g->nu - 1) * p->ang[3 * kk] : 0.0) +
                         ((c & 2) ? (g->nv - 1) * p->ang[3 * kk + 1] : 0.0);
        if (!(t >= -0.999 && t < g->n_s - 0.001)) inside = false;
      }
    }
    p->splat_max_terms = max_terms;
    p->splat_checked = inside ? 0 : 1;
  }
  p->chunks.clear();
  for (int kk = 0; kk < K;) {
    int colmajor = std::fabs(p->ang[3 * kk + 1]) > std::fabs(p->ang[3 * kk]) ? 1 : 0;
    int e = kk;
    while (e < K && e - kk < kc && (std::fabs(p->ang[3 * e + 1]) > std::fabs(p->ang[3 * e]) ? 1 : 0) == colmajor) ++e;
    p->chunks.insert(p->chunks.end(), {kk, e - kk, colmajor, 0});
    kk = e;
  }
  p->n_chunks = (int)p->chunks.size() / 4;

  p->vf.assign(4 * n, 0.f);
  p->rmax2.assign(n, 0.f);
  p->frame.assign(12 * n, 0.0);
  p->proj.assign(12 * n, 0.0);
  for (int v = 0; v < n; ++v)
    for (int c = 0; c < 3; ++c) {
      p->frame[12 * v + c] = views[v].src[c];
      p->frame[12 * v + 3 + c] = views[v].det_center[c];
      p->frame[12 * v + 6 + c] = views[v].ex[c];
      p->frame[12 * v + 9 + c] = views[v].ey[c];
    }
  std::vector<double> zrel(n);
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
    p->vf[4 * v] = (float)D;
    p->vf[4 * v + 1] = (float)(dot3(w.tangent, w.ex) / (four_pi2 * D));
    p->vf[4 * v + 2] = (float)(dot3(w.tangent, w.ey) / (four_pi2 * D));
    p->vf[4 * v + 3] = (float)(dot3(w.tangent, lz) / (four_pi2 * D * D));
    double rel0[3];
    for (int c = 0; c < 3; ++c) rel0[c] = X0[c] - w.src[c];
    double* P = &p->proj[12 * v];
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
    p->rmax2[v] = (float)((D / umin) * (D / umin) * (1.0 + 1e-6));
    zrel[v] = std::fabs(P[2]) / (umin / D);   // largest relative change of den per voxel step in z
    max_cell_terms = std::max(max_cell_terms, cell_terms_bound(g, w, D, X0, umax));
    P[7] = dot3(rel0, w.ex) / g->du + 0.5 * (g->nu - 1) * dn0;
    P[11] = dot3(rel0, w.ey) / g->dv + 0.5 * (g->nv - 1) * dn0;
  }

  if (max_cell_terms > (double)kMaxCellTerms)
    return fail(err, DC_ENOTSUP,
                "up to " + std::to_string((long long)max_cell_terms) +
                    " voxel centres can project into one detector cell (limit " + std::to_string(kMaxCellTerms) +
                    "); the detector is too coarse for the voxel grid");
  p->cone_max_terms = (int)std::max(1.0, max_cell_terms);
  // widest and tallest backprojection block footprint (same box rule as the kernel)
  // -> the row pitch of the staged footprint and how many of its rows each thread
  // stages per view
  {
    const int B[3] = {ks.bp_bx, ks.bp_by, ks.bp_bz};
    const int nb[3] = {(g->nx + B[0] - 1) / B[0], (g->ny + B[1] - 1) / B[1], (g->nz + B[2] - 1) / B[2]};
    double worst_w = 0, worst_h = 0;
    for (int v = 0; v < n; ++v) {
      const double* P = &p->proj[12 * v];
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
              imin = std::min(imin, iu);
              imax = std::max(imax, iu);
              jmin = std::min(jmin, jv);
              jmax = std::max(jmax, jv);
            }
            // kernel box: [floor(min)-1, floor(max)+2], plus slack for float rounding
            const double bw = std::floor(imax) - std::floor(imin) + 5, bh = std::floor(jmax) - std::floor(jmin) + 5;
            worst_w = std::max(worst_w, bw);
            worst_h = std::max(worst_h, bh);
          }
    }
    // rows are staged PITCH pixels apart, each by PITCH / 64 whole waves, so a wave's
    // row index is uniform; kBPThreads / PITCH rows per pass, STAGE passes
    p->bp_pitch = worst_w <= 64 ? 64 : worst_w <= 128 ? 128 : 0;
    p->bp_stage = 0;
    if (p->bp_pitch > 0) {
      const int need = (int)std::ceil(worst_h / (double)(ks.bp_threads() / p->bp_pitch));
      p->bp_stage = need <= 4 ? 4 : need <= 8 ? 8 : need <= 12 ? 12 : need <= 16 ? 16 : 0;
    }
    if (p->bp_stage == 0) p->bp_pitch = 0;
  }
  // Form of the cone kernels, decided per sample (so a batched plan computes what
  // each scan's own plan does).  den = U/D and num_u free of z on every view: a
  // voxel column keeps one u and one weight per view, formed once per column.
  // Otherwise, if den changes by at most 5e-4 of itself per voxel step, 1/den
  // along a 16-voxel segment is its quadratic Taylor polynomial about the
  // segment's middle, whose remainder is below (7.5 x 5e-4)^3 = 5.3e-8 (float
  // rounding), and replaces the per-voxel reciprocal.
  p->cone_form.assign(n_samples, kConeZinv);
  for (int smp = 0; smp < n_samples; ++smp) {
    bool zinv = true;
    double worst = 0.0;
    for (int v = first[smp]; v < first[smp + 1]; ++v) {
      zinv = zinv && p->proj[12 * v + 2] == 0.0 && p->proj[12 * v + 6] == 0.0;
      worst = std::max(worst, zrel[v]);
    }
    p->cone_form[smp] = zinv ? kConeZinv : worst <= 5e-4 ? kConeQuadratic : kConeGeneral;
  }
  return DC_OK;
}

}  // namespace dc
