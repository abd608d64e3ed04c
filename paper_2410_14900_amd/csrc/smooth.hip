// Gaussian smoothing of the learned redundancy weight (paper Sec. 3.1: a Gaussian
// filter layer after the weight layer) and its exact transpose.
//
//   Ms = G_mu G_s M   per view,   (G x)[i] = sum_{t=-r..r} w_t x[mirror(i + t)],
//   w_t = exp(-t^2 / (2 sigma^2)) normalised over t = -r..r,
//   mirror(m) = -m (m < 0), m, 2(n-1) - m (m > n-1)   (edge sample not repeated).
//
// Each 1D pass stages its lines in LDS with r-sample halos and every thread
// produces kOB consecutive outputs of a line from a sliding register window, so
// one LDS read feeds kOB FMAs.  The forward pass fills the halos by mirroring.
// The transpose of one pass is
//   gx[j] = C(j) + [j > 0] C(-j) + [j < n-1] C(2(n-1) - j),
//   C(c)  = sum_t w_t gy[c - t]  over 0 <= c - t < n,
// i.e. the same convolution with zero halos (the symmetric w makes it a
// correlation), plus the two mirrored terms, which only the r outputs at each end
// receive and which a short second loop adds.  Every workgroup reads all it
// writes before its barrier and workgroups touch disjoint lines, so both passes
// may run in place.
#include <cmath>

#include "dc_internal.h"

namespace dc {

static constexpr int kOB = 4;        // consecutive outputs per thread
static constexpr int kSmCols = 16;   // s-columns per workgroup of the mu pass

// kOB outputs y[j0 .. j0+kOB) of sum_t w_|t| v(j + t), where v(m) = lds[(m + r) * stride]
__device__ __forceinline__ void conv_run(const float* __restrict__ lds, int stride, const float* __restrict__ w,
                                         int r, int j0, float* acc) {
  float win[kOB];
#pragma unroll
  for (int k = 0; k < kOB; ++k) {
    win[k] = lds[(j0 + k) * stride];   // v(j0 + k - r), the window for t = -r
    acc[k] = 0.f;
  }
  for (int t = -r; t <= r; ++t) {
    const float wt = w[t < 0 ? -t : t];
#pragma unroll
    for (int k = 0; k < kOB; ++k) acc[k] = fmaf(wt, win[k], acc[k]);
#pragma unroll
    for (int k = 0; k < kOB - 1; ++k) win[k] = win[k + 1];
    win[kOB - 1] = lds[(j0 + kOB + t + r) * stride];   // v(j0 + kOB - 1 + t + 1), halo covers it
  }
}

// the mirrored terms of the transpose for output j of a line of length n held
// (without halo offset) at g(m) = lds[(m + r) * stride]
__device__ __forceinline__ float mirror_terms(const float* __restrict__ lds, int stride, const float* __restrict__ w,
                                              int r, int n, int j) {
  auto C = [&](int c) {
    float a = 0.f;
    const int lo = max(-r, c - n + 1), hi = min(r, c);
    for (int t = lo; t <= hi; ++t) a = fmaf(w[t < 0 ? -t : t], lds[(c - t + r) * stride], a);
    return a;
  };
  float a = 0.f;
  if (j > 0 && j <= r) a += C(-j);
  if (j < n - 1 && j >= n - 1 - r) a += C(2 * (n - 1) - j);
  return a;
}

// s-pass: one workgroup per (mu row, view); lds = taps [r + 1] then the line [ns + 2r + kOB]
template <bool ADJ>
__global__ __launch_bounds__(256) void k_smooth_s(const float* in, float* out, int n_theta, int ns, GaussTaps tp,
                                                  int r, int v0) {
  extern __shared__ float sm[];
  float* w = sm;
  float* line = sm + r + 1;
  const size_t base = ((size_t)(v0 + blockIdx.y) * n_theta + blockIdx.x) * ns;
  for (int q = threadIdx.x; q <= r; q += blockDim.x) w[q] = tp.w[q];
  for (int q = threadIdx.x; q < ns + 2 * r + kOB; q += blockDim.x) {
    int m = q - r;
    float v = 0.f;
    if (!ADJ) {
      if (m < 0) m = -m;
      else if (m > ns - 1) m = 2 * (ns - 1) - m;
      if (m >= 0 && m < ns) v = in[base + m];   // the kOB tail beyond the halo is never weighted
    } else if (m >= 0 && m < ns) {
      v = in[base + m];
    }
    line[q] = v;
  }
  __syncthreads();
  for (int j0 = threadIdx.x * kOB; j0 < ns; j0 += blockDim.x * kOB) {
    float acc[kOB];
    conv_run(line, 1, w, r, j0, acc);
#pragma unroll
    for (int k = 0; k < kOB; ++k) {
      const int j = j0 + k;
      if (j < ns) out[base + j] = ADJ ? acc[k] + mirror_terms(line, 1, w, r, ns, j) : acc[k];
    }
  }
}

// mu-pass: one workgroup per (block of kSmCols s-columns, view);
// lds = taps [r + 1] then the columns [n_theta + 2r + kOB][kSmCols]
template <bool ADJ>
__global__ __launch_bounds__(256) void k_smooth_mu(const float* in, float* out, int n_theta, int ns, GaussTaps tp,
                                                   int r, int v0) {
  extern __shared__ float sm[];
  float* w = sm;
  float* cols = sm + r + 1;
  const int c0 = blockIdx.x * kSmCols;
  const size_t vbase = (size_t)(v0 + blockIdx.y) * n_theta * ns;
  const int rows = n_theta + 2 * r + kOB;
  for (int q = threadIdx.x; q <= r; q += blockDim.x) w[q] = tp.w[q];
  for (int q = threadIdx.x; q < rows * kSmCols; q += blockDim.x) {
    const int rr = q / kSmCols, c = q - rr * kSmCols;
    int k = rr - r;
    float v = 0.f;
    if (!ADJ) {
      if (k < 0) k = -k;
      else if (k > n_theta - 1) k = 2 * (n_theta - 1) - k;
    }
    if (k >= 0 && k < n_theta && c0 + c < ns) v = in[vbase + (size_t)k * ns + c0 + c];
    cols[q] = v;
  }
  __syncthreads();
  const int nblk = (n_theta + kOB - 1) / kOB;
  for (int q = threadIdx.x; q < nblk * kSmCols; q += blockDim.x) {
    const int jb = q / kSmCols, c = q - jb * kSmCols;
    const int j0 = jb * kOB;
    float acc[kOB];
    conv_run(cols + c, kSmCols, w, r, j0, acc);
#pragma unroll
    for (int k = 0; k < kOB; ++k) {
      const int j = j0 + k;
      if (j < n_theta && c0 + c < ns)
        out[vbase + (size_t)j * ns + c0 + c] =
            ADJ ? acc[k] + mirror_terms(cols + c, kSmCols, w, r, n_theta, j) : acc[k];
    }
  }
}

size_t smooth_mu_lds_bytes(int n_theta, int r) {
  return (size_t)(r + 1 + (n_theta + 2 * r + kOB) * kSmCols) * sizeof(float);
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
  const size_t lds_s = (size_t)(r + 1 + S + 2 * r + kOB) * sizeof(float);
  const size_t lds_m = (size_t)(r + 1 + (K + 2 * r + kOB) * kSmCols) * sizeof(float);
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
