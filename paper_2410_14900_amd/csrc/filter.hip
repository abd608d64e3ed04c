// Shift-variant filtering in the sinogram domain (paper eqs. 7, 10, 11):
//
//   Q = D R,   P = W Q,   H = D P,     W = M c_geo  (ANALYTIC)  or  W = M  (RAW)
//   c_geo(k, m) = -| t.n_mu / (4 pi^2 D) + s_m t.l_z / (4 pi^2 D^2) |
//
// D is the zero-padded central difference along s.  The adjoint gives
// GP = D^T GH = -D GH, GM = GP Q c_geo and GR = D^T (W GP).
// One workgroup filters one sinogram row (v, k): the row is read from HBM once
// into LDS, both differences and the weight are applied there, and the result
// is written once -- the stage is bound by its 12 bytes/bin of HBM traffic.
#include "dc_internal.h"

namespace dc {

__device__ __forceinline__ float cgeo_row(const float4 vf, const float2 cs) {
  return vf.y * cs.x + vf.z * cs.y;   // t.n_mu / (4 pi^2 D)
}

template <typename TR, typename TH>
__global__ __launch_bounds__(256) void k_filter(const TR* __restrict__ R, const float* __restrict__ M,
                                                TH* __restrict__ H, KGrid g,
                                                const float4* __restrict__ viewf,
                                                const float2* __restrict__ trig, int raw, int v0) {
  extern __shared__ float sh[];
  float* r = sh;            // [ns]
  float* pw = sh + g.n_s;   // [ns]
  const int ns = g.n_s;
  const int k = blockIdx.x, v = v0 + blockIdx.y;
  const size_t row = ((size_t)v * g.n_theta + k) * ns;
  for (int m = threadIdx.x; m < ns; m += blockDim.x) r[m] = to_f32(R[row + m]);
  __syncthreads();
  const float4 vf = viewf[v];
  const float a = cgeo_row(vf, trig[k]);
  const float inv2ds = 0.5f / g.ds;
  const float s0 = -0.5f * (ns - 1) * g.ds;
  for (int m = threadIdx.x; m < ns; m += blockDim.x) {
    float rp = (m + 1 < ns) ? r[m + 1] : 0.f;
    float rm = (m > 0) ? r[m - 1] : 0.f;
    float w = M[row + m];
    if (!raw) w *= -fabsf(fmaf(fmaf((float)m, g.ds, s0), vf.w, a));
    pw[m] = w * (rp - rm) * inv2ds;
  }
  __syncthreads();
  for (int m = threadIdx.x; m < ns; m += blockDim.x) {
    float pp = (m + 1 < ns) ? pw[m + 1] : 0.f;
    float pm = (m > 0) ? pw[m - 1] : 0.f;
    H[row + m] = from_f32<TH>((pp - pm) * inv2ds);
  }
}

template <typename TH, typename TR>
__global__ __launch_bounds__(256) void k_filter_adj(const TH* __restrict__ GH, const TR* __restrict__ R,
                                                    const float* __restrict__ M, float* __restrict__ GM,
                                                    int acc, float* __restrict__ GR, KGrid g,
                                                    const float4* __restrict__ viewf,
                                                    const float2* __restrict__ trig, int raw, int v0) {
  extern __shared__ float sh[];
  float* gh = sh;            // [ns]
  float* r = sh + g.n_s;     // [ns]
  float* gq = sh + 2 * g.n_s;  // [ns]
  const int ns = g.n_s;
  const int k = blockIdx.x, v = v0 + blockIdx.y;
  const size_t row = ((size_t)v * g.n_theta + k) * ns;
  for (int m = threadIdx.x; m < ns; m += blockDim.x) {
    gh[m] = to_f32(GH[row + m]);
    r[m] = to_f32(R[row + m]);
  }
  __syncthreads();
  const float4 vf = viewf[v];
  const float a = cgeo_row(vf, trig[k]);
  const float inv2ds = 0.5f / g.ds;
  const float s0 = -0.5f * (ns - 1) * g.ds;
  for (int m = threadIdx.x; m < ns; m += blockDim.x) {
    float gp = (((m > 0) ? gh[m - 1] : 0.f) - ((m + 1 < ns) ? gh[m + 1] : 0.f)) * inv2ds;
    float q = (((m + 1 < ns) ? r[m + 1] : 0.f) - ((m > 0) ? r[m - 1] : 0.f)) * inv2ds;
    float c = raw ? 1.f : -fabsf(fmaf(fmaf((float)m, g.ds, s0), vf.w, a));
    if (GM) {
      float gm = gp * q * c;
      GM[row + m] = acc ? GM[row + m] + gm : gm;
    }
    if (GR) gq[m] = M[row + m] * c * gp;
  }
  if (GR) {
    __syncthreads();
    for (int m = threadIdx.x; m < ns; m += blockDim.x)
      GR[row + m] = (((m > 0) ? gq[m - 1] : 0.f) - ((m + 1 < ns) ? gq[m + 1] : 0.f)) * inv2ds;
  }
}

hipError_t launch_filter(const Plan& p, const void* R, dc_dtype tR, const float* M, int raw, void* H,
                         dc_dtype tH, int v0, int nv, hipStream_t s) {
  dim3 grid(p.kg.n_theta, nv);
  const size_t lds = 2 * (size_t)p.kg.n_s * sizeof(float);
  return by_dtype(tR, [&](auto tr) {
    using TR = decltype(tr);
    return by_dtype(tH, [&](auto th) {
      using TH = decltype(th);
      hipLaunchKernelGGL((k_filter<TR, TH>), grid, dim3(256), lds, s, (const TR*)R, M, (TH*)H, p.kg,
                         (const float4*)p.d_view, (const float2*)p.d_trig, raw, v0);
      return hipGetLastError();
    });
  });
}

hipError_t launch_filter_adjoint(const Plan& p, const void* GH, dc_dtype tH, const void* R, dc_dtype tR,
                                 const float* M, int raw, float* GM, int acc, float* GR, int v0, int nv,
                                 hipStream_t s) {
  dim3 grid(p.kg.n_theta, nv);
  const size_t lds = 3 * (size_t)p.kg.n_s * sizeof(float);
  return by_dtype(tH, [&](auto th) {
    using TH = decltype(th);
    return by_dtype(tR, [&](auto tr) {
      using TR = decltype(tr);
      hipLaunchKernelGGL((k_filter_adj<TH, TR>), grid, dim3(256), lds, s, (const TH*)GH, (const TR*)R, M, GM, acc,
                         GR, p.kg, (const float4*)p.d_view, (const float2*)p.d_trig, raw, v0);
      return hipGetLastError();
    });
  });
}

}  // namespace dc
