// Structural similarity of two volumes (the SSIM term of the training loss, eq. 13)
// and its gradient w.r.t. the first volume.
//
// Standard definition in 3D: window moments mu_x = G*x, mu_y = G*y, E[x^2], E[y^2],
// E[xy] with the normalised Gaussian window G (sigma 1.5, 11 taps per axis) at the
// positions where the whole window lies inside the volume ("valid" grid),
//   S = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_xx + s_yy + C2)),
// SSIM = mean S.  The gradient spreads the per-position derivatives of S w.r.t.
// (mu_x, E[x^2], E[xy]) back over the windows (the transposed valid convolution,
// zero outside) and combines them as (T0 + 2 x T1 + y T2) / N.
//
// Work is three separable passes each way over a caller-provided workspace; the
// mean is reduced in a fixed order (per-block partial sums, then one block), so
// results are bit-reproducible.
#include <cmath>

#include "dc_internal.h"

namespace dc {

static constexpr int kSsR = 5, kSsT = 2 * kSsR + 1;
struct SsimWindow {
  float w[kSsT];
};

static SsimWindow ssim_window() {
  SsimWindow s{};
  double sum = 0.0, v[kSsT];
  for (int t = 0; t < kSsT; ++t) sum += (v[t] = std::exp(-0.5 * ((t - kSsR) / 1.5) * ((t - kSsR) / 1.5)));
  for (int t = 0; t < kSsT; ++t) s.w[t] = (float)(v[t] / sum);
  return s;
}

// first pass along z: the five moments from x and y.  out [5][nz-10][ny][nx]
__global__ __launch_bounds__(256) void k_ss_moments_z(const float* __restrict__ x, const float* __restrict__ y,
                                                      float* __restrict__ out, int nz, int ny, int nx,
                                                      SsimWindow W) {
  const size_t plane = (size_t)ny * nx, n_out = (size_t)(nz - 2 * kSsR) * plane;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n_out; q += (size_t)gridDim.x * blockDim.x) {
    float a[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < kSsT; ++t) {
      const float xv = x[q + t * plane], yv = y[q + t * plane], wt = W.w[t];
      a[0] = fmaf(wt, xv, a[0]);
      a[1] = fmaf(wt, yv, a[1]);
      a[2] = fmaf(wt, xv * xv, a[2]);
      a[3] = fmaf(wt, yv * yv, a[3]);
      a[4] = fmaf(wt, xv * yv, a[4]);
    }
#pragma unroll
    for (int f = 0; f < 5; ++f) out[f * n_out + q] = a[f];
  }
}

// one 1D pass over NF fields of shape [d0][d1][d2] (in) along axis 1 or 2:
// forward = valid convolution (that axis shrinks by 10), transpose = full
// convolution of the zero-padded input (that axis grows by 10)
template <int NF, int AXIS, bool TRANSPOSE>
__global__ __launch_bounds__(256) void k_ss_pass(const float* __restrict__ in, float* __restrict__ out, int d0,
                                                 int d1, int d2, SsimWindow W) {
  const int o1 = AXIS == 1 ? (TRANSPOSE ? d1 + 2 * kSsR : d1 - 2 * kSsR) : d1;
  const int o2 = AXIS == 2 ? (TRANSPOSE ? d2 + 2 * kSsR : d2 - 2 * kSsR) : d2;
  const size_t n_in = (size_t)d0 * d1 * d2, n_out = (size_t)d0 * o1 * o2;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n_out; q += (size_t)gridDim.x * blockDim.x) {
    const int i2 = (int)(q % o2);
    const size_t r = q / o2;
    const int i1 = (int)(r % o1), i0 = (int)(r / o1);
    float a[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) a[f] = 0.f;
#pragma unroll
    for (int t = 0; t < kSsT; ++t) {
      // forward: in index = out index + t;  transpose: in index = out index - t
      int j1 = i1, j2 = i2;
      if (AXIS == 1) j1 = TRANSPOSE ? i1 - t : i1 + t;
      else j2 = TRANSPOSE ? i2 - t : i2 + t;
      if (TRANSPOSE && ((unsigned)j1 >= (unsigned)d1 || (unsigned)j2 >= (unsigned)d2)) continue;
      const size_t src = ((size_t)i0 * d1 + j1) * d2 + j2;
#pragma unroll
      for (int f = 0; f < NF; ++f) a[f] = fmaf(W.w[t], in[f * n_in + src], a[f]);
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) out[f * n_out + q] = a[f];
  }
}

// transpose along z of the three derivative fields, combined into the gradient:
// grad = (T0 + 2 x T1 + y T2) / N, where T_f = G_z^T(in_f), in_f [3][nz-10][ny][nx]
__global__ __launch_bounds__(256) void k_ss_grad_z(const float* __restrict__ in, const float* __restrict__ x,
                                                   const float* __restrict__ y, float* __restrict__ grad, int nz,
                                                   int ny, int nx, float invN, SsimWindow W) {
  const size_t plane = (size_t)ny * nx, n_in = (size_t)(nz - 2 * kSsR) * plane, n = (size_t)nz * plane;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
    const int iz = (int)(q / plane);
    const size_t rest = q - (size_t)iz * plane;
    float a[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < kSsT; ++t) {
      const int jz = iz - t;
      if ((unsigned)jz >= (unsigned)(nz - 2 * kSsR)) continue;
      const size_t src = (size_t)jz * plane + rest;
#pragma unroll
      for (int f = 0; f < 3; ++f) a[f] = fmaf(W.w[t], in[f * n_in + src], a[f]);
    }
    grad[q] = (a[0] + 2.f * x[q] * a[1] + y[q] * a[2]) * invN;
  }
}

// SSIM map on the valid grid: S summed per block (fixed-order tree) into part[],
// and, when WANT_GRAD, the derivative fields d[3][n] = (dS/dmu_x, dS/dE[x^2], dS/dE[xy])
template <bool WANT_GRAD>
__global__ __launch_bounds__(256) void k_ss_map(const float* __restrict__ mom, size_t n, float C1, float C2,
                                                double* __restrict__ part, float* __restrict__ d) {
  __shared__ double red[256];
  double s = 0.0;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
    const float mx = mom[q], my = mom[n + q], exx = mom[2 * n + q], eyy = mom[3 * n + q], exy = mom[4 * n + q];
    const float A1 = 2.f * mx * my + C1, A2 = 2.f * (exy - mx * my) + C2;
    const float B1 = mx * mx + my * my + C1, B2 = (exx - mx * mx) + (eyy - my * my) + C2;
    const float inv = 1.f / (B1 * B2);
    const float S = A1 * A2 * inv;
    s += (double)S;
    if (WANT_GRAD) {
      d[q] = 2.f * my * (A2 - A1) * inv - 2.f * mx * S * (1.f / B1 - 1.f / B2);
      d[n + q] = -S / B2;
      d[2 * n + q] = 2.f * A1 * inv;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_ss_mean(const double* __restrict__ part, int nb, double invN,
                                                 float* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = (float)(red[0] * invN);
}

static constexpr int kSsMapBlocks = 1024;

size_t ssim_workspace_bytes(int nz, int ny, int nx) {
  const size_t a = (size_t)(nz - 2 * kSsR) * ny * nx;   // after the z pass
  // two ping-pong buffers of 5 fields (the largest intermediate) plus the partial sums
  return 2 * 5 * a * sizeof(float) + kSsMapBlocks * sizeof(double) + 256;
}

static int blocks_for(size_t n) { return (int)std::min<size_t>(8192, (n + 255) / 256); }

hipError_t launch_ssim(const float* x, const float* y, int nz, int ny, int nx, float L, float* ssim, float* grad,
                       void* work, hipStream_t s) {
  const SsimWindow W = ssim_window();
  const int vz = nz - 2 * kSsR, vy = ny - 2 * kSsR, vx = nx - 2 * kSsR;
  const size_t a = (size_t)vz * ny * nx, b = (size_t)vz * vy * nx, c = (size_t)vz * vy * vx;
  float* buf0 = (float*)work;
  float* buf1 = buf0 + 5 * a;
  double* part = (double*)(buf1 + 5 * a);
  const float C1 = (0.01f * L) * (0.01f * L), C2 = (0.03f * L) * (0.03f * L);
  hipLaunchKernelGGL(k_ss_moments_z, dim3(blocks_for(a)), dim3(256), 0, s, x, y, buf0, nz, ny, nx, W);
  hipLaunchKernelGGL((k_ss_pass<5, 1, false>), dim3(blocks_for(b)), dim3(256), 0, s, buf0, buf1, vz, ny, nx, W);
  hipLaunchKernelGGL((k_ss_pass<5, 2, false>), dim3(blocks_for(c)), dim3(256), 0, s, buf1, buf0, vz, vy, nx, W);
  // buf0 now holds the 5 moments on the valid grid [5][vz][vy][vx]
  if (grad) {
    hipLaunchKernelGGL(k_ss_map<true>, dim3(kSsMapBlocks), dim3(256), 0, s, buf0, c, C1, C2, part, buf1);
    hipLaunchKernelGGL(k_ss_mean, dim3(1), dim3(256), 0, s, part, kSsMapBlocks, 1.0 / (double)c, ssim);
    // spread the 3 derivative fields back: x, then y, then z (combined with x and y)
    hipLaunchKernelGGL((k_ss_pass<3, 2, true>), dim3(blocks_for((size_t)vz * vy * nx)), dim3(256), 0, s, buf1,
                       buf0, vz, vy, vx, W);
    hipLaunchKernelGGL((k_ss_pass<3, 1, true>), dim3(blocks_for(a)), dim3(256), 0, s, buf0, buf1, vz, vy, nx, W);
    hipLaunchKernelGGL(k_ss_grad_z, dim3(blocks_for((size_t)nz * ny * nx)), dim3(256), 0, s, buf1, x, y, grad, nz,
                       ny, nx, (float)(1.0 / (double)c), W);
  } else {
    hipLaunchKernelGGL(k_ss_map<false>, dim3(kSsMapBlocks), dim3(256), 0, s, buf0, c, C1, C2, part, nullptr);
    hipLaunchKernelGGL(k_ss_mean, dim3(1), dim3(256), 0, s, part, kSsMapBlocks, 1.0 / (double)c, ssim);
  }
  return hipGetLastError();
}

}  // namespace dc
