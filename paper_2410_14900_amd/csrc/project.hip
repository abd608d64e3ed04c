// Cone-beam forward projector for making projection data from a voxel volume:
// Siddon's exact line integral of the piecewise-constant voxel function (R. L.
// Siddon, Med. Phys. 12(2), 1985) along the segment from the source to each
// detector pixel centre, g = |p1 - p0| * sum_k (alpha_{k+1} - alpha_k) f(voxel_k).
//
// One thread per ray walks the voxels incrementally: from the entry parameter it
// repeatedly steps across the nearest of the next x, y or z boundary planes,
// which visits the same segments as merging and sorting all plane crossings.
// The walk runs in float64 (on this GPU a float64 FMA issues at the float32
// rate of non-packed code), every index is checked before a volume read, and the
// number of steps is capped at nx + ny + nz + 3, so every wave exits.
#include <cmath>

#include "dc_internal.h"

namespace dc {

struct VoxelBox {
  double lo[3], v[3];   // first boundary plane and voxel size per axis (x, y, z)
  double du, dv;        // detector pitch
  int n[3];
};

__global__ __launch_bounds__(256) void k_project(const float* __restrict__ vol, float* __restrict__ g, KGrid kg,
                                                 const double* __restrict__ frame, const int* __restrict__ first,
                                                 int n_samples, int v0, VoxelBox box) {
  const int v = v0 + blockIdx.y;
  const int npix = kg.nu * kg.nv;
  const int pix = blockIdx.x * blockDim.x + threadIdx.x;
  if (pix >= npix) return;
  const int j = pix / kg.nu, i = pix - j * kg.nu;
  int smp = 0;                                   // sample (scan) of view v
  while (smp + 1 < n_samples && first[smp + 1] <= v) ++smp;
  const float* f = vol + (size_t)smp * box.n[0] * box.n[1] * box.n[2];
  const double* F = frame + 12 * v;
  const double x = (i - 0.5 * (kg.nu - 1)) * box.du, y = (j - 0.5 * (kg.nv - 1)) * box.dv;
  double p0[3], d[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    p0[a] = F[a];
    d[a] = F[3 + a] + x * F[6 + a] + y * F[9 + a] - F[a];
  }
  double lo = 0.0, hi = 1.0;
  bool miss = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double P0 = box.lo[a], P1 = box.lo[a] + box.n[a] * box.v[a];
    if (d[a] != 0.0) {
      const double t0 = (P0 - p0[a]) / d[a], t1 = (P1 - p0[a]) / d[a];
      lo = fmax(lo, fmin(t0, t1));
      hi = fmin(hi, fmax(t0, t1));
    } else if (p0[a] < P0 || p0[a] > P1) {
      miss = true;
    }
  }
  double acc = 0.0;
  if (!miss && lo < hi) {
    int idx[3], step[3];
    double next[3], dal[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double pe = p0[a] + lo * d[a];
      int k = (int)floor((pe - box.lo[a]) / box.v[a]);
      k = min(max(k, 0), box.n[a] - 1);
      idx[a] = k;
      if (d[a] > 0.0) {
        next[a] = (box.lo[a] + (k + 1) * box.v[a] - p0[a]) / d[a];
        step[a] = 1;
        dal[a] = box.v[a] / d[a];
      } else if (d[a] < 0.0) {
        next[a] = (box.lo[a] + k * box.v[a] - p0[a]) / d[a];
        step[a] = -1;
        dal[a] = -box.v[a] / d[a];
      } else {
        next[a] = 1e300;
        step[a] = 0;
        dal[a] = 0.0;
      }
    }
    double cur = lo;
    const int cap = box.n[0] + box.n[1] + box.n[2] + 3;
    for (int it = 0; it < cap; ++it) {
      const int a = next[0] <= next[1] ? (next[0] <= next[2] ? 0 : 2) : (next[1] <= next[2] ? 1 : 2);
      const double t = fmin(next[a], hi);
      acc += fmax(t - cur, 0.0) * (double)f[((size_t)idx[2] * box.n[1] + idx[1]) * box.n[0] + idx[0]];
      cur = t;
      if (t >= hi) break;
      idx[a] += step[a];
      if ((unsigned)idx[a] >= (unsigned)box.n[a]) break;
      next[a] += dal[a];
    }
  }
  const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  g[(size_t)v * npix + pix] = (float)(acc * len);
}

hipError_t launch_project(const Plan& p, const float* vol, float* g, int v0, int nv, hipStream_t s) {
  const dc_grid& G = p.grid;
  VoxelBox box;
  box.n[0] = G.nx; box.n[1] = G.ny; box.n[2] = G.nz;
  box.v[0] = G.vx; box.v[1] = G.vy; box.v[2] = G.vz;
  box.lo[0] = G.ox - 0.5 * G.nx * G.vx;
  box.lo[1] = G.oy - 0.5 * G.ny * G.vy;
  box.lo[2] = G.oz - 0.5 * G.nz * G.vz;
  box.du = G.du;
  box.dv = G.dv;
  const int npix = G.nu * G.nv;
  hipLaunchKernelGGL(k_project, dim3((npix + 255) / 256, nv), dim3(256), 0, s, vol, g, p.kg, p.d_frame, p.d_first,
                     p.n_samples, v0, box);
  return hipGetLastError();
}

}  // namespace dc
