// 2D parallel-beam Radon pair on each detector image (paper eqs. 7, 8, 11):
//
//   splat : out[k][m] = scale * sum_p w(p) img(p) Lambda(t_pk - m)     (A2d and the detector Radon)
//   interp: out(p)    = scale * w(p) sum_k lerp(rows[k], t_pk)          (A2d^T and the transposed A2d)
//
// with t_pk = i A_k + j B_k + C_k the fractional s-bin of pixel p=(i,j) on angle
// mu_k, Lambda the hat function and w the optional cosine weight D/sqrt(x^2+y^2+D^2).
// The two are exact transposes of each other for equal scales.
#include "dc_internal.h"

namespace dc {

// ------------------------------------------------------------------ splat
// One workgroup owns one view and a chunk of <= kc angles whose sinogram rows
// live in LDS.  Every pixel of the view is read once per chunk and deposits its
// two hat-function weights with LDS float atomics; rows are then written out
// once (no global atomics).  For angles closer to the detector rows the lanes of
// a wave walk along i, otherwise along j, so that neighbouring lanes fall into
// different bins and LDS atomics rarely collide.
//
// The fractional bin t reaches ~n_s, where a float32 ulp is 1e-4 bin, so t is
// formed in float64 (full-rate FMA on CDNA) and only the fraction is rounded.
template <typename Tin, typename Tout, bool WCOS>
__global__ __launch_bounds__(256) void k_splat(const Tin* __restrict__ img, Tout* __restrict__ out, KGrid g,
                                               const int4* __restrict__ chunks,
                                               const double* __restrict__ angd,
                                               const float4* __restrict__ viewf, float scale, int v0) {
  extern __shared__ float rows[];
  __shared__ double sA[16], sB[16], sC[16];
  const int4 ch = chunks[blockIdx.x];
  const int v = v0 + blockIdx.y;
  const int k0 = ch.x, kn = ch.y, colmajor = ch.z;
  const int ns = g.n_s;
  for (int q = threadIdx.x; q < kn * ns; q += blockDim.x) rows[q] = 0.f;
  if (threadIdx.x < kn) {
    const int k = k0 + threadIdx.x;
    sA[threadIdx.x] = angd[3 * k];
    sB[threadIdx.x] = angd[3 * k + 1];
    sC[threadIdx.x] = angd[3 * k + 2];
  }
  __syncthreads();
  const int npix = g.nu * g.nv;
  const Tin* im = img + (size_t)v * npix;
  const float D = viewf[v].x;
  for (int q = threadIdx.x; q < npix; q += blockDim.x) {
    int i, j;
    if (colmajor) {
      i = q / g.nv;
      j = q - i * g.nv;
    } else {
      j = q / g.nu;
      i = q - j * g.nu;
    }
    float x = to_f32(im[j * g.nu + i]);
    if (WCOS) {
      float xu = (i - g.cu) * g.du, yv = (j - g.cv) * g.dv;
      x *= D * rsqrtf(fmaf(xu, xu, fmaf(yv, yv, D * D)));
    }
    const double di = (double)i, dj = (double)j;
    for (int kk = 0; kk < kn; ++kk) {
      double t = fma(di, sA[kk], fma(dj, sB[kk], sC[kk]));
      double fl = floor(t);
      int m = (int)fl;
      float w1 = x * (float)(t - fl);
      float w0 = x - w1;
      float* r = rows + kk * ns;
      if ((unsigned)m < (unsigned)ns) atomicAdd(r + m, w0);
      if ((unsigned)(m + 1) < (unsigned)ns) atomicAdd(r + m + 1, w1);
    }
  }
  __syncthreads();
  Tout* o = out + ((size_t)v * g.n_theta + k0) * ns;
  for (int q = threadIdx.x; q < kn * ns; q += blockDim.x) o[q] = from_f32<Tout>(scale * rows[q]);
}

// ----------------------------------------------------------------- interp
// One workgroup owns a 32 x 16 pixel tile of one view (256 threads, 2 pixels
// each).  Angles are processed in chunks of 32: for each angle the tile's s-range
// (plus margins) of the row is staged in LDS as (value, next - value) pairs, so a
// linear-interpolation tap is one 8-byte LDS read and one FMA.  Tile-local
// fractional positions are derived from float64 per-(tile, angle) offsets, which
// keeps them below ~40 bins and their float32 rounding below 4e-6 bins.
static constexpr int kTX = 32, kTY = 16, kKC = 32;

template <typename Tin, typename Tout, bool WCOS>
__global__ __launch_bounds__(256) void k_interp(const Tin* __restrict__ rows, Tout* __restrict__ out, KGrid g,
                                                const double* __restrict__ angd,
                                                const float4* __restrict__ angf,
                                                const float4* __restrict__ viewf, float scale, int v0, int wl,
                                                int tiles_u) {
  extern __shared__ float2 win[];
  __shared__ float sOff[kKC], sA[kKC], sB[kKC];
  __shared__ int sW0[kKC];
  const int v = v0 + blockIdx.y;
  const int tu = blockIdx.x % tiles_u, tv = blockIdx.x / tiles_u;
  const int i0 = tu * kTX, j0 = tv * kTY;
  const int tx = threadIdx.x & (kTX - 1), ty = threadIdx.x / kTX;  // ty in [0, 8)
  const int ns = g.n_s;
  const Tin* rv = rows + (size_t)v * g.n_theta * ns;
  float acc0 = 0.f, acc1 = 0.f;
  for (int k0 = 0; k0 < g.n_theta; k0 += kKC) {
    const int kn = min(kKC, g.n_theta - k0);
    if (threadIdx.x < kn) {
      const int k = k0 + threadIdx.x;
      const double A = angd[3 * k], B = angd[3 * k + 1], C = angd[3 * k + 2];
      const double t00 = C + i0 * A + j0 * B;
      const double tmin = t00 + fmin(0.0, (kTX - 1) * A) + fmin(0.0, (kTY - 1) * B);
      const int w0 = (int)floor(tmin) - 1;
      sW0[threadIdx.x] = w0;
      sOff[threadIdx.x] = (float)(t00 - w0);
      sA[threadIdx.x] = (float)A;
      sB[threadIdx.x] = (float)B;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kn * wl; q += blockDim.x) {
      const int kk = q / wl, e = q - kk * wl;
      const int m = sW0[kk] + e;
      const Tin* r = rv + (size_t)(k0 + kk) * ns;
      float a = ((unsigned)m < (unsigned)ns) ? to_f32(r[m]) : 0.f;
      float b = ((unsigned)(m + 1) < (unsigned)ns) ? to_f32(r[m + 1]) : 0.f;
      win[q] = make_float2(a, b - a);
    }
    __syncthreads();
    const float fx = (float)tx, fy = (float)ty;
    for (int kk = 0; kk < kn; ++kk) {
      const float A = sA[kk], B = sB[kk];
      const float t = fmaf(fx, A, fmaf(fy, B, sOff[kk]));
      const float t2 = fmaf(8.f, B, t);
      const int m = (int)t, m2 = (int)t2;
      const float2 p = win[kk * wl + m], p2 = win[kk * wl + m2];
      acc0 += fmaf(t - (float)m, p.y, p.x);
      acc1 += fmaf(t2 - (float)m2, p2.y, p2.x);
    }
    __syncthreads();
  }
  const float D = viewf[v].x;
  const int i = i0 + tx;
  Tout* o = out + (size_t)v * g.nu * g.nv;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int j = j0 + ty + 8 * h;
    if (i < g.nu && j < g.nv) {
      float val = scale * (h ? acc1 : acc0);
      if (WCOS) {
        float xu = (i - g.cu) * g.du, yv = (j - g.cv) * g.dv;
        val *= D * rsqrtf(fmaf(xu, xu, fmaf(yv, yv, D * D)));
      }
      o[j * g.nu + i] = from_f32<Tout>(val);
    }
  }
}

// --------------------------------------------------------------- dispatch

hipError_t launch_splat(const Plan& p, const void* img, dc_dtype t_in, bool wcos, float scale, void* out,
                        dc_dtype t_out, int v0, int nv, hipStream_t s) {
  const size_t lds = (size_t)p.splat_kc * p.kg.n_s * sizeof(float);
  dim3 grid(p.n_chunks, nv);
  return by_dtype(t_in, [&](auto tin) {
    using Tin = decltype(tin);
    return by_dtype(t_out, [&](auto tout) {
      using Tout = decltype(tout);
      if (wcos)
        hipLaunchKernelGGL((k_splat<Tin, Tout, true>), grid, dim3(256), lds, s, (const Tin*)img, (Tout*)out, p.kg,
                           p.d_chunks, p.d_ang, (const float4*)p.d_view, scale, v0);
      else
        hipLaunchKernelGGL((k_splat<Tin, Tout, false>), grid, dim3(256), lds, s, (const Tin*)img, (Tout*)out, p.kg,
                           p.d_chunks, p.d_ang, (const float4*)p.d_view, scale, v0);
      return hipGetLastError();
    });
  });
}

hipError_t launch_interp(const Plan& p, const void* rows, dc_dtype t_in, bool wcos, float scale, void* out,
                         dc_dtype t_out, int v0, int nv, hipStream_t s) {
  const int tiles_u = (p.kg.nu + kTX - 1) / kTX, tiles_v = (p.kg.nv + kTY - 1) / kTY;
  const size_t lds = (size_t)kKC * p.interp_wl * sizeof(float2);
  dim3 grid(tiles_u * tiles_v, nv);
  return by_dtype(t_in, [&](auto tin) {
    using Tin = decltype(tin);
    return by_dtype(t_out, [&](auto tout) {
      using Tout = decltype(tout);
      if (wcos)
        hipLaunchKernelGGL((k_interp<Tin, Tout, true>), grid, dim3(256), lds, s, (const Tin*)rows, (Tout*)out,
                           p.kg, p.d_ang, (const float4*)p.d_angf, (const float4*)p.d_view, scale, v0,
                           p.interp_wl, tiles_u);
      else
        hipLaunchKernelGGL((k_interp<Tin, Tout, false>), grid, dim3(256), lds, s, (const Tin*)rows, (Tout*)out,
                           p.kg, p.d_ang, (const float4*)p.d_angf, (const float4*)p.d_view, scale, v0,
                           p.interp_wl, tiles_u);
      return hipGetLastError();
    });
  });
}

}  // namespace dc
