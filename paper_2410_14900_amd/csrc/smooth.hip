// Gaussian smoothing of the learned redundancy weight (paper Sec. 3.1: a Gaussian
// filter layer after the weight layer) and its exact transpose.
//
//   Ms = G_mu G_s M   per view,   (G x)[i] = sum_{t=-r..r} w_t x[mirror(i + t)],
//   w_t = exp(-t^2 / (2 sigma^2)) normalised over t = -r..r,
//   mirror(m) = -m (m < 0), m, 2(n-1) - m (m > n-1)   (edge sample not repeated).
//
// Each 1D pass stages its lines in LDS.  The transpose of one pass gathers
//   gx[j] = C(j) + [j > 0] C(-j) + [j < n-1] C(2(n-1) - j),
//   C(c)  = sum_t w_t gy[c - t]  over 0 <= c - t < n,
// the three ways mirror(i + t) can equal j.  Every workgroup reads all it writes
// before its barrier and workgroups touch disjoint lines, so both passes may run
// in place.
#include <cmath>

#include "dc_internal.h"

namespace dc {

// s-pass: one workgroup per (mu row, view)
template <bool ADJ>
__global__ __launch_bounds__(256) void k_smooth_s(const float* in, float* out, int n_theta, int ns, GaussTaps tp,
                                                  int r, int v0) {
  extern __shared__ float line[];   // forward: [ns + 2r] with mirrored halos; transpose: [ns]
  const size_t base = ((size_t)(v0 + blockIdx.y) * n_theta + blockIdx.x) * ns;
  const int len = ADJ ? ns : ns + 2 * r;
  for (int q = threadIdx.x; q < len; q += blockDim.x) {
    int m = ADJ ? q : q - r;
    if (m < 0) m = -m;
    else if (m > ns - 1) m = 2 * (ns - 1) - m;
    line[q] = in[base + m];
  }
  __syncthreads();
  for (int j = threadIdx.x; j < ns; j += blockDim.x) {
    float acc = 0.f;
    if (!ADJ) {
      for (int t = -r; t <= r; ++t) acc = fmaf(tp.w[t < 0 ? -t : t], line[j + r + t], acc);
    } else {
      auto C = [&](int c) {
        float a = 0.f;
        const int lo = max(-r, c - ns + 1), hi = min(r, c);
        for (int t = lo; t <= hi; ++t) a = fmaf(tp.w[t < 0 ? -t : t], line[c - t], a);
        return a;
      };
      acc = C(j);
      if (j > 0 && j <= r) acc += C(-j);
      if (j < ns - 1 && j >= ns - 1 - r) acc += C(2 * (ns - 1) - j);
    }
    out[base + j] = acc;
  }
}

// mu-pass: one workgroup per (block of kSmCols s-columns, view)
static constexpr int kSmCols = 16;

template <bool ADJ>
__global__ __launch_bounds__(256) void k_smooth_mu(const float* in, float* out, int n_theta, int ns, GaussTaps tp,
                                                   int r, int v0) {
  extern __shared__ float cols[];   // [rows][kSmCols], rows = n_theta + 2r (forward) or n_theta
  const int c0 = blockIdx.x * kSmCols;
  const size_t vbase = (size_t)(v0 + blockIdx.y) * n_theta * ns;
  const int rows = ADJ ? n_theta : n_theta + 2 * r;
  for (int q = threadIdx.x; q < rows * kSmCols; q += blockDim.x) {
    const int rr = q / kSmCols, c = q - rr * kSmCols;
    int k = ADJ ? rr : rr - r;
    if (k < 0) k = -k;
    else if (k > n_theta - 1) k = 2 * (n_theta - 1) - k;
    cols[q] = c0 + c < ns ? in[vbase + (size_t)k * ns + c0 + c] : 0.f;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < n_theta * kSmCols; q += blockDim.x) {
    const int j = q / kSmCols, c = q - j * kSmCols;
    float acc = 0.f;
    if (!ADJ) {
      for (int t = -r; t <= r; ++t) acc = fmaf(tp.w[t < 0 ? -t : t], cols[(j + r + t) * kSmCols + c], acc);
    } else {
      auto C = [&](int cc) {
        float a = 0.f;
        const int lo = max(-r, cc - n_theta + 1), hi = min(r, cc);
        for (int t = lo; t <= hi; ++t) a = fmaf(tp.w[t < 0 ? -t : t], cols[(cc - t) * kSmCols + c], a);
        return a;
      };
      acc = C(j);
      if (j > 0 && j <= r) acc += C(-j);
      if (j < n_theta - 1 && j >= n_theta - 1 - r) acc += C(2 * (n_theta - 1) - j);
    }
    if (c0 + c < ns) out[vbase + (size_t)j * ns + c0 + c] = acc;
  }
}

GaussTaps gauss_taps(double sigma, int r) {
  GaussTaps tp{};
  double sum = 0.0;
  for (int t = -r; t <= r; ++t) sum += std::exp(-0.5 * (t / sigma) * (t / sigma));
  for (int t = 0; t <= r; ++t) tp.w[t] = (float)(std::exp(-0.5 * (t / sigma) * (t / sigma)) / sum);
  return tp;
}

hipError_t launch_smooth(const Plan& p, const float* in, float* out, double sigma, int r, bool adjoint, int v0,
                         int nv, hipStream_t s) {
  const int K = p.kg.n_theta, S = p.kg.n_s;
  const GaussTaps tp = gauss_taps(sigma, r);
  const dim3 gs(K, nv), gm((S + kSmCols - 1) / kSmCols, nv);
  const size_t lds_s = (size_t)(adjoint ? S : S + 2 * r) * sizeof(float);
  const size_t lds_m = (size_t)(adjoint ? K : K + 2 * r) * kSmCols * sizeof(float);
  if (!adjoint) {
    // G_mu G_s M: the s-pass into out, then the mu-pass in place
    hipLaunchKernelGGL(k_smooth_s<false>, gs, dim3(256), lds_s, s, in, out, K, S, tp, r, v0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_smooth_mu<false>, gm, dim3(256), lds_m, s, out, out, K, S, tp, r, v0);
  } else {
    // (G_mu G_s)^T = G_s^T G_mu^T
    hipLaunchKernelGGL(k_smooth_mu<true>, gm, dim3(256), lds_m, s, in, out, K, S, tp, r, v0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_smooth_s<true>, gs, dim3(256), lds_s, s, out, out, K, S, tp, r, v0);
  }
  return hipGetLastError();
}

}  // namespace dc
