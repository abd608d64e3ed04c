// Smooth Crofton redundancy weight (eq. 9; Defrise & Clack's smooth replacement
// of 1/n, Sec. 2.4) on the Radon grid of every view:
//
//   M(theta, tau_v) = w(tau_v) / sum_alpha w(tau_alpha),  w(tau) = |a'(tau).theta|^m c(tau),
//
// the sum running over the orbit parameters whose source point lies in the plane
// {p : p.theta = a(tau_v).theta}.  One thread owns one (view, angle, bin) entry,
// all in float64.  Circles, arcs and lines are intersected in closed form.  On a
// sinusoid the plane function F(tau) = a(tau).theta - d is sampled on a fixed grid
// (a table of points built once per call), each sign change between neighbouring
// samples brackets a crossing, and 80 bisection steps on the analytic curve
// refine it.  The scan skips samples that cannot change sign: |F'| <= |a'| <= L =
// R sqrt(1 + (phi_max f)^2), so from a sample with |F| > L k h (h the sample step)
// the next k samples keep its sign (a margin of 1e-6 covers the rounding of the
// table and of the dot products); every sign change the full scan would see is
// still found, in the same bracket.  Brackets are kept per thread in LDS and
// refined after the scan, so the lanes of a wave bisect together instead of one
// bracket at a time.
#include <cmath>

#include "dc_internal.h"

namespace dc {

static constexpr int kCrofMaxSegs = 16;
static constexpr int kCrofBrackets = 16;    // brackets kept per thread and sinusoid segment
static constexpr double kCrofSkipMargin = 1e-6;   // mm: far above the rounding of F on the table
static constexpr int kCrofBisect = 80;
static constexpr double kTwoPi = 6.283185307179586;   // 2 pi rounded to double

struct CrofSeg {
  int kind, start, count, closed;
  double p0, p1, phi_max, freq;
  double lo, hi;        // parameters of the first and last view
  long long samp;       // sinusoid: offset of its points in the table ([n][3] doubles)
  int n_samp;
};
struct CrofArgs {
  CrofSeg seg[kCrofMaxSegs];
  int n_seg;
  double R, taper, c_floor, ds;
  int m_exp;
};

__device__ __forceinline__ void seg_point(const CrofSeg& s, double R, double tau, double* a) {
  double st, ct;
  sincos(tau, &st, &ct);
  if (s.kind == DC_SEG_CIRCLE) {
    a[0] = R * ct; a[1] = R * st; a[2] = 0.0;
  } else if (s.kind == DC_SEG_ARC) {
    a[0] = R * ct; a[1] = 0.0; a[2] = R * st;
  } else if (s.kind == DC_SEG_LINE) {
    a[0] = R; a[1] = 0.0; a[2] = tau;
  } else {
    double sp, cp;
    sincos(s.phi_max * cos(s.freq * tau), &sp, &cp);
    a[0] = R * (cp * ct); a[1] = R * (cp * st); a[2] = R * sp;
  }
}

// a'(tau) times the segment's per-view parameter step
__device__ __forceinline__ void seg_tangent(const CrofSeg& s, double R, double tau, double* t) {
  double st, ct;
  sincos(tau, &st, &ct);
  if (s.kind == DC_SEG_CIRCLE) {
    t[0] = s.p1 * (-R * st); t[1] = s.p1 * (R * ct); t[2] = 0.0;
  } else if (s.kind == DC_SEG_ARC) {
    t[0] = s.p1 * (-R * st); t[1] = 0.0; t[2] = s.p1 * (R * ct);
  } else if (s.kind == DC_SEG_LINE) {
    t[0] = 0.0; t[1] = 0.0; t[2] = s.p1;
  } else {
    const double f = s.freq, ph = s.phi_max * cos(f * tau), dph = -s.phi_max * f * sin(f * tau);
    double sp, cp;
    sincos(ph, &sp, &cp);
    t[0] = s.p1 * (R * (-sp * dph * ct - cp * st));
    t[1] = s.p1 * (R * (-sp * dph * st + cp * ct));
    t[2] = s.p1 * (R * (cp * dph));
  }
}

__device__ __forceinline__ double seg_taper(const CrofSeg& s, double tau, double taper, double c_floor) {
  if (s.closed) return 1.0;
  const double u = (tau - s.lo) / (s.hi - s.lo);
  const double e = fmin(u, 1.0 - u) / taper;
  const double ramp = e < 1.0 ? 0.5 - 0.5 * cos(M_PI * fmin(fmax(e, 0.0), 1.0)) : 1.0;
  return c_floor + (1.0 - c_floor) * ramp;
}

__device__ __forceinline__ double ipow(double x, int m) {
  double r = x;
  for (int i = 1; i < m; ++i) r *= x;
  return r;
}

__device__ __forceinline__ double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

__device__ __forceinline__ double seg_weight(const CrofSeg& s, const CrofArgs& A, double tau, const double* th) {
  double t[3];
  seg_tangent(s, A.R, tau, t);
  return ipow(fabs(dot3(t, th)), A.m_exp) * seg_taper(s, tau, A.taper, A.c_floor);
}

// x mod y with the sign of y (y > 0), as Python's float modulo
__device__ __forceinline__ double pymod(double x, double y) {
  double r = fmod(x, y);
  if (r != 0.0 && r < 0.0) r += y;
  return r;
}

// 80 bisection steps on the analytic curve over [a, b] (F(a) <= 0 given by fa_nonpos)
__device__ double bisect(const CrofSeg& s, double R, const double* th, double d, double a, double b, bool fa_nonpos) {
  for (int it = 0; it < kCrofBisect; ++it) {
    const double mid = 0.5 * (a + b);
    double p[3];
    seg_point(s, R, mid, p);
    const double fm = dot3(p, th) - d;
    if ((fm <= 0.0) == fa_nonpos) {
      a = mid;
      fa_nonpos = fm <= 0.0;
    } else {
      b = mid;
    }
  }
  return 0.5 * (a + b);
}

__device__ __forceinline__ int sgn(double x) { return (x > 0.0) - (x < 0.0); }

// sinusoid sample points tau_j = p0 + (j + 1/2) 2 pi / n, table [n][3]
__global__ void k_crofton_samples(CrofArgs A, double* __restrict__ table) {
  const int si = blockIdx.y;
  const CrofSeg& s = A.seg[si];
  if (s.kind != DC_SEG_SINUSOID) return;
  const double step = kTwoPi / s.n_samp;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < s.n_samp; j += gridDim.x * blockDim.x) {
    double p[3];
    seg_point(s, A.R, s.p0 + (j + 0.5) * step, p);
    double* o = table + s.samp + 3ll * j;
    o[0] = p[0]; o[1] = p[1]; o[2] = p[2];
  }
}

__global__ __launch_bounds__(256) void k_crofton(CrofArgs A, const double* __restrict__ frame,
                                                 const double* __restrict__ table, float* __restrict__ M,
                                                 int n_theta, int n_s, int v0) {
  __shared__ int sBr[kCrofBrackets][256];
  const int v = v0 + blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_theta * n_s) return;   // no barriers below: every thread works alone
  const int k = e / n_s, m = e - k * n_s;
  // view frame and the normal theta of this (angle, bin)
  const double* F = frame + 12 * v;
  const double lx[3] = {F[6], F[7], F[8]}, ly[3] = {F[9], F[10], F[11]};
  const double lz[3] = {lx[1] * ly[2] - lx[2] * ly[1], lx[2] * ly[0] - lx[0] * ly[2], lx[0] * ly[1] - lx[1] * ly[0]};
  const double rel[3] = {F[0] - F[3], F[1] - F[4], F[2] - F[5]};
  const double D = dot3(rel, lz);
  const double mu = k * M_PI / n_theta;
  const double sm = (m - (n_s - 1) / 2.0) * A.ds;
  double cm, sn;
  sincos(mu, &sn, &cm);
  const double hyp = hypot(sm, D);
  double th[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) th[c] = (D * (cm * lx[c] + sn * ly[c]) + sm * lz[c]) / hyp;
  // the view's own orbit point and parameter
  int sv = 0;
  while (sv + 1 < A.n_seg && A.seg[sv + 1].start <= v) ++sv;
  const CrofSeg& S = A.seg[sv];
  const double tau_v = S.p0 + (v - S.start) * S.p1;
  double av[3];
  seg_point(S, A.R, tau_v, av);
  const double d = dot3(av, th);

  double den = 0.0;
  int count = 0;
  for (int si = 0; si < A.n_seg; ++si) {
    const CrofSeg& s = A.seg[si];
    if (s.kind == DC_SEG_CIRCLE || s.kind == DC_SEG_ARC) {
      const double c1 = th[0], c2 = s.kind == DC_SEG_CIRCLE ? th[1] : th[2];
      const double rho = A.R * hypot(c1, c2);
      if (rho == 0.0 || fabs(d) > rho * (1.0 + 1e-12)) continue;
      const double base = atan2(c2, c1);
      const double ac = acos(fmax(-1.0, fmin(1.0, d / rho)));
      for (int c = 0; c < (ac > 0.0 ? 2 : 1); ++c) {
        double tau = c == 0 ? base + ac : base - ac;
        if (s.kind == DC_SEG_CIRCLE) {
          if (s.closed) {
            tau = pymod(tau - s.p0, kTwoPi) + s.p0;
          } else {
            // the covered parameters only; the window opens 1e-12 below the first
            // view's, so a crossing at the first source point survives rounding
            tau = pymod(tau - s.lo + 1e-12, kTwoPi) + s.lo - 1e-12;
            if (!(tau <= s.hi + 1e-12)) continue;
            tau = fmin(fmax(tau, s.lo), s.hi);
          }
        } else {
          tau = pymod(tau + M_PI, kTwoPi) - M_PI;
          if (!(tau >= s.lo - 1e-12 && tau <= s.hi + 1e-12)) continue;
          tau = fmin(fmax(tau, s.lo), s.hi);
        }
        den += seg_weight(s, A, tau, th);
        ++count;
      }
    } else if (s.kind == DC_SEG_LINE) {
      if (th[2] == 0.0) continue;
      const double z = (d - A.R * th[0]) / th[2];
      if (!(z >= s.lo - 1e-12 && z <= s.hi + 1e-12)) continue;
      den += seg_weight(s, A, z, th);
      ++count;
    } else {
      // sinusoid: scan the sampled plane function for sign changes
      const int n = s.n_samp;
      const double step = kTwoPi / n;
      const double* P = table + s.samp;
      // L h, with a relative margin for the rounding of L itself
      const double lh = A.R * sqrt(1.0 + (s.phi_max * s.freq) * (s.phi_max * s.freq)) * step * (1.0 + 1e-9);
      auto sample = [&](int j) { return P[3ll * j] * th[0] + P[3ll * j + 1] * th[1] + P[3ll * j + 2] * th[2] - d; };
      int nbr = 0;
      const double f_first = sample(0);
      double f_prev = f_first;   // the last sample looked at (or one of the same sign)
      int j = 0;
      while (j + 1 < n) {
        // samples j+1 .. j+skip keep the sign of f_prev: no bracket among them
        const double room = (fabs(f_prev) - kCrofSkipMargin) / lh;
        const int skip = room >= 1.0 ? (int)fmin(room, (double)(n - 1 - j)) : 0;
        j += skip;
        if (j + 1 >= n) break;   // the last sample has f_prev's sign
        ++j;
        const double f = sample(j);
        if (sgn(f_prev) * sgn(f) <= 0) {
          // bracket [tau_{j-1}, tau_j]; sample j-1 has f_prev's sign
          if (nbr < kCrofBrackets) {
            sBr[nbr][threadIdx.x] = (j - 1) * 2 + (f_prev <= 0.0 ? 1 : 0);
          } else {
            const double r = bisect(s, A.R, th, d, s.p0 + (j - 1 + 0.5) * step, s.p0 + (j + 0.5) * step,
                                    f_prev <= 0.0);
            den += seg_weight(s, A, r, th);
          }
          ++nbr;
        }
        f_prev = f;
      }
      // refine the kept brackets (lanes bisect together)
      const int kept = min(nbr, kCrofBrackets);
      for (int b = 0; b < kept; ++b) {
        const int code = sBr[b][threadIdx.x];
        const int j = code >> 1;
        const double r = bisect(s, A.R, th, d, s.p0 + (j + 0.5) * step, s.p0 + (j + 1 + 0.5) * step, code & 1);
        den += seg_weight(s, A, r, th);
      }
      count += nbr;
      // the interval across the end of the turn
      if (sgn(f_prev) * sgn(f_first) < 0) {
        const double r = bisect(s, A.R, th, d, s.p0 + (n - 1 + 0.5) * step, s.p0 + 0.5 * step + kTwoPi,
                                f_prev <= 0.0);
        den += seg_weight(s, A, r, th);
        ++count;
      }
    }
  }
  double tv[3];
  seg_tangent(S, A.R, tau_v, tv);
  const double num = ipow(fabs(dot3(tv, th)), A.m_exp) * seg_taper(S, tau_v, A.taper, A.c_floor);
  const double tol = 1e-18 * ipow(sqrt(dot3(tv, tv)), A.m_exp);
  const double val = den > tol ? num / den : 1.0 / (double)max(count, 1);
  M[((size_t)v * n_theta + k) * n_s + m] = (float)val;
}

// -------------------------------------------------------------------- host
static bool build_args(const Plan& p, const dc_orbit_segment* segs, int n_segs, double sid, int m_exp, double taper,
                       double c_floor, int fine, CrofArgs* A, size_t* table_bytes) {
  *A = CrofArgs{};
  A->n_seg = n_segs;
  A->R = sid;
  A->taper = taper;
  A->c_floor = c_floor;
  A->ds = p.grid.ds;
  A->m_exp = m_exp;
  long long off = 0;
  for (int i = 0; i < n_segs; ++i) {
    CrofSeg& c = A->seg[i];
    const dc_orbit_segment& s = segs[i];
    c.kind = s.kind; c.start = s.start; c.count = s.count; c.closed = s.closed;
    c.p0 = s.p0; c.p1 = s.p1; c.phi_max = s.phi_max; c.freq = s.freq;
    c.lo = s.p0 + 0 * s.p1;
    c.hi = s.p0 + (s.count - 1) * s.p1;
    c.samp = off;
    c.n_samp = 0;
    if (s.kind == DC_SEG_SINUSOID) {
      c.n_samp = fine * s.count;
      off += 3ll * c.n_samp;
    }
  }
  *table_bytes = (size_t)off * sizeof(double);
  return true;
}

size_t crofton_workspace_bytes(const dc_orbit_segment* segs, int n_segs, int fine) {
  size_t b = 0;
  for (int i = 0; i < n_segs; ++i)
    if (segs[i].kind == DC_SEG_SINUSOID) b += (size_t)3 * fine * segs[i].count * sizeof(double);
  return b + 256;
}

int crofton_max_segments() { return kCrofMaxSegs; }

hipError_t launch_crofton(const Plan& p, const dc_orbit_segment* segs, int n_segs, double sid, int m_exp,
                          double taper, double c_floor, int fine, float* M, int v0, int nv, void* work,
                          hipStream_t s) {
  CrofArgs A;
  size_t tb = 0;
  build_args(p, segs, n_segs, sid, m_exp, taper, c_floor, fine, &A, &tb);
  double* table = (double*)(((uintptr_t)work + 255) & ~(uintptr_t)255);
  if (tb > 0) {
    hipLaunchKernelGGL(k_crofton_samples, dim3(64, n_segs), dim3(256), 0, s, A, table);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int entries = p.kg.n_theta * p.kg.n_s;
  hipLaunchKernelGGL(k_crofton, dim3((entries + 255) / 256, nv), dim3(256), 0, s, A, p.d_frame, table, M,
                     p.kg.n_theta, p.kg.n_s, v0);
  return hipGetLastError();
}

}  // namespace dc
