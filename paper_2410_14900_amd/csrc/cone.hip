// Cone-beam backprojection (paper eq. 5 with the detector weight of eq. 11 folded
// in) and its exact transpose, the cone-beam forward projection:
//
//   f(x)       (+)= sum_v (D/U)^2 sum_{i,j} gF_v[j][i] Lambda(i* - i) Lambda(j* - j)
//   GgF_v[j][i]  = sum_x (D/U)^2 Gf(x)    Lambda(i* - i) Lambda(j* - j)
//
// with the per-view projective map i* = num_u/den, j* = num_v/den, den = U/D,
// all affine in the voxel index (float64 table built by the plan).
//
// Work mapping: a thread owns one (x, y) voxel column segment of kZC voxels and
// walks it in z; lanes of a wave are consecutive x, so volume reads and writes
// are coalesced.  For every view the thread forms its column's projection
// coefficients in float64 relative to an integer detector origin near the
// column's projection, so the float32 per-voxel coordinates stay small and
// their rounding far below 1e-5 pixel.
#include "dc_internal.h"

namespace dc {

static constexpr int kBX = 64, kBY = 4, kZC = 16;

struct ColumnMap {
  float den, dden;   // den = U/D at the segment start and its z step
  float lu, ldu;     // num_u - iu0 den and its z step
  float lv, ldv;     // num_v - jv0 den and its z step
  int iu0, jv0;
};

__device__ __forceinline__ ColumnMap column_map(const double* __restrict__ P, int ix, int iy, int iz0) {
  const double den = fma((double)ix, P[0], fma((double)iy, P[1], fma((double)iz0, P[2], P[3])));
  const double nu = fma((double)ix, P[4], fma((double)iy, P[5], fma((double)iz0, P[6], P[7])));
  const double nv = fma((double)ix, P[8], fma((double)iy, P[9], fma((double)iz0, P[10], P[11])));
  ColumnMap c;
  const float rden = 1.0f / (float)den;
  c.iu0 = (int)floorf((float)nu * rden);
  c.jv0 = (int)floorf((float)nv * rden);
  c.den = (float)den;
  c.dden = (float)P[2];
  c.lu = (float)fma(-(double)c.iu0, den, nu);
  c.ldu = (float)fma(-(double)c.iu0, P[2], P[6]);
  c.lv = (float)fma(-(double)c.jv0, den, nv);
  c.ldv = (float)fma(-(double)c.jv0, P[2], P[10]);
  return c;
}

template <typename T>
__device__ __forceinline__ float tap(const T* __restrict__ img, int i, int j, int nu, int nv) {
  return ((unsigned)i < (unsigned)nu && (unsigned)j < (unsigned)nv) ? to_f32(img[j * nu + i]) : 0.f;
}

template <typename T>
__global__ __launch_bounds__(256) void k_cone_bp(const T* __restrict__ gF, float* __restrict__ f, KGrid g,
                                                 const double* __restrict__ proj, int acc_in, int relu, int v0,
                                                 int nv) {
  const int ix = blockIdx.x * kBX + threadIdx.x;
  const int iy = blockIdx.y * kBY + threadIdx.y;
  const int iz0 = blockIdx.z * kZC;
  float acc[kZC];
#pragma unroll
  for (int z = 0; z < kZC; ++z) acc[z] = 0.f;
  const size_t npix = (size_t)g.nu * g.nv;
  for (int v = v0; v < v0 + nv; ++v) {
    const ColumnMap c = column_map(proj + 12 * v, ix, iy, iz0);
    const T* img = gF + (size_t)v * npix;
#pragma unroll
    for (int z = 0; z < kZC; ++z) {
      const float den = fmaf((float)z, c.dden, c.den);
      const float r = __builtin_amdgcn_rcpf(den);
      const float u = fmaf((float)z, c.ldu, c.lu) * r;
      const float w = fmaf((float)z, c.ldv, c.lv) * r;
      const float fu0 = floorf(u), fw0 = floorf(w);
      const float fu = u - fu0, fw = w - fw0;
      const int i = c.iu0 + (int)fu0, j = c.jv0 + (int)fw0;
      const float a00 = tap(img, i, j, g.nu, g.nv), a01 = tap(img, i + 1, j, g.nu, g.nv);
      const float a10 = tap(img, i, j + 1, g.nu, g.nv), a11 = tap(img, i + 1, j + 1, g.nu, g.nv);
      const float top = fmaf(fu, a01 - a00, a00), bot = fmaf(fu, a11 - a10, a10);
      acc[z] = fmaf(r * r, fmaf(fw, bot - top, top), acc[z]);
    }
  }
  if (ix >= g.nx || iy >= g.ny) return;
#pragma unroll
  for (int z = 0; z < kZC; ++z) {
    const int iz = iz0 + z;
    if (iz < g.nz) {
      float* o = f + ((size_t)iz * g.ny + iy) * g.nx + ix;
      float val = acc_in ? *o + acc[z] : acc[z];
      *o = relu ? fmaxf(val, 0.f) : val;
    }
  }
}

__global__ void k_fill_zero(float* __restrict__ p, size_t n) {
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x)
    p[q] = 0.f;
}

// Scatter form of the transpose: each voxel adds its four weighted taps to the
// view's detector image with global float atomics.
__global__ __launch_bounds__(256) void k_cone_fp_scatter(const float* __restrict__ Gf,
                                                         const float* __restrict__ f_relu,
                                                         float* __restrict__ GgF, KGrid g,
                                                         const double* __restrict__ proj, int v0, int nv) {
  const int ix = blockIdx.x * kBX + threadIdx.x;
  const int iy = blockIdx.y * kBY + threadIdx.y;
  const int iz0 = blockIdx.z * kZC;
  float gv[kZC];
  const bool col_ok = ix < g.nx && iy < g.ny;
#pragma unroll
  for (int z = 0; z < kZC; ++z) {
    const int iz = iz0 + z;
    float x = 0.f;
    if (col_ok && iz < g.nz) {
      const size_t o = ((size_t)iz * g.ny + iy) * g.nx + ix;
      x = Gf[o];
      if (f_relu && !(f_relu[o] > 0.f)) x = 0.f;
    }
    gv[z] = x;
  }
  const size_t npix = (size_t)g.nu * g.nv;
  for (int v = v0; v < v0 + nv; ++v) {
    const ColumnMap c = column_map(proj + 12 * v, ix, iy, iz0);
    float* img = GgF + (size_t)v * npix;
#pragma unroll
    for (int z = 0; z < kZC; ++z) {
      if (gv[z] == 0.f) continue;
      const float den = fmaf((float)z, c.dden, c.den);
      const float r = __builtin_amdgcn_rcpf(den);
      const float u = fmaf((float)z, c.ldu, c.lu) * r;
      const float w = fmaf((float)z, c.ldv, c.lv) * r;
      const float fu0 = floorf(u), fw0 = floorf(w);
      const float fu = u - fu0, fw = w - fw0;
      const int i = c.iu0 + (int)fu0, j = c.jv0 + (int)fw0;
      const float s = r * r * gv[z];
      const float b0 = s * (1.f - fw), b1 = s * fw;
      const bool i0ok = (unsigned)i < (unsigned)g.nu, i1ok = (unsigned)(i + 1) < (unsigned)g.nu;
      if ((unsigned)j < (unsigned)g.nv) {
        if (i0ok) atomicAdd(img + j * g.nu + i, b0 * (1.f - fu));
        if (i1ok) atomicAdd(img + j * g.nu + i + 1, b0 * fu);
      }
      if ((unsigned)(j + 1) < (unsigned)g.nv) {
        if (i0ok) atomicAdd(img + (j + 1) * g.nu + i, b1 * (1.f - fu));
        if (i1ok) atomicAdd(img + (j + 1) * g.nu + i + 1, b1 * fu);
      }
    }
  }
}

hipError_t launch_cone_bp(const Plan& p, const void* gF, dc_dtype tF, float* f, int acc, int relu, int v0, int nv,
                          hipStream_t s) {
  dim3 grid((p.kg.nx + kBX - 1) / kBX, (p.kg.ny + kBY - 1) / kBY, (p.kg.nz + kZC - 1) / kZC);
  return by_dtype(tF, [&](auto t) {
    using T = decltype(t);
    hipLaunchKernelGGL((k_cone_bp<T>), grid, dim3(kBX, kBY), 0, s, (const T*)gF, f, p.kg, p.d_proj, acc, relu, v0,
                       nv);
    return hipGetLastError();
  });
}

hipError_t launch_cone_fp(const Plan& p, const float* Gf, const float* f_relu, void* GgF, dc_dtype tF, int v0,
                          int nv, hipStream_t s) {
  if (tF != DC_F32) return hipErrorNotSupported;
  float* out = (float*)GgF + (size_t)v0 * p.kg.nu * p.kg.nv;
  const size_t n = (size_t)nv * p.kg.nu * p.kg.nv;
  hipLaunchKernelGGL(k_fill_zero, dim3(1024), dim3(256), 0, s, out, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 grid((p.kg.nx + kBX - 1) / kBX, (p.kg.ny + kBY - 1) / kBY, (p.kg.nz + kZC - 1) / kZC);
  hipLaunchKernelGGL(k_cone_fp_scatter, grid, dim3(kBX, kBY), 0, s, Gf, f_relu, (float*)GgF, p.kg, p.d_proj, v0,
                     nv);
  return hipGetLastError();
}

}  // namespace dc
