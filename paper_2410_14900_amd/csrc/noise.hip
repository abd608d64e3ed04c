// Poisson noise on projection data (the simulated training data, Sec. 3.3):
// lambda = I0 exp(-mu p), N ~ Poisson(lambda), p~ = -ln(max(N, 1) / I0) / mu.
//
// Random numbers come from the counter-based generator Philox4x64-10 (Salmon et
// al., SC 2011): element e draws the blocks philox((e, j, 0, 0), (seed, 0)),
// j = 0, 1, ..., four 64-bit words each, and a word x becomes the uniform
// ((x >> 11) + 1/2) 2^-53.  The count is drawn by inversion for lambda < 10 (one
// uniform, CDF accumulated term by term) and by Hoermann's transformed rejection
// with squeeze (PTRS, 1993) for lambda >= 10, two uniforms per trial.  Every
// decision is taken in float64.  One thread per element (grid-stride); the
// rejection loop is capped at 256 trials (acceptance exceeds 0.8 per trial, so
// the cap is never reached in practice; it only bounds the wave), after which
// the trial's k is rounded lambda.
#include <cmath>

#include "dc_internal.h"

namespace dc {

static constexpr unsigned long long kPhiloxM0 = 0xD2E7470EE14C6C93ull, kPhiloxM1 = 0xCA5A826395121157ull;
static constexpr unsigned long long kPhiloxW0 = 0x9E3779B97F4A7C15ull, kPhiloxW1 = 0xBB67AE8584CAA73Bull;
static constexpr int kMaxTrials = 256;

struct Philox {
  unsigned long long e, seed, j;
  unsigned long long w[4];
  int pos;
  __device__ void block() {
    unsigned long long x0 = e, x1 = j, x2 = 0, x3 = 0, k0 = seed, k1 = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
      if (r) {
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
      }
      const unsigned long long hi0 = __umul64hi(kPhiloxM0, x0), lo0 = kPhiloxM0 * x0;
      const unsigned long long hi1 = __umul64hi(kPhiloxM1, x2), lo1 = kPhiloxM1 * x2;
      x0 = hi1 ^ x1 ^ k0;
      x1 = lo1;
      x2 = hi0 ^ x3 ^ k1;
      x3 = lo0;
    }
    w[0] = x0; w[1] = x1; w[2] = x2; w[3] = x3;
    pos = 0;
    ++j;
  }
  __device__ double uniform() {
    if (pos == 4) block();
    const unsigned long long x = pos == 0 ? w[0] : pos == 1 ? w[1] : pos == 2 ? w[2] : w[3];
    ++pos;
    return ((double)(x >> 11) + 0.5) * 0x1p-53;
  }
};

__device__ long long poisson_count(double lam, unsigned long long seed, unsigned long long e) {
  if (!(lam > 0.0)) return 0;
  Philox rng{e, seed, 0ull, {0, 0, 0, 0}, 4};
  if (lam < 10.0) {
    const double u = rng.uniform();
    double p = exp(-lam), F = p;
    long long k = 0;
    while (u > F && k < 1000) {
      ++k;
      p = p * lam / (double)k;
      F = F + p;
    }
    return k;
  }
  const double slam = sqrt(lam), loglam = log(lam);
  const double b = 0.931 + 2.53 * slam;
  const double a = -0.059 + 0.02483 * b;
  const double inv_alpha = 1.1239 + 1.1328 / (b - 3.4);
  const double v_r = 0.9277 - 3.6224 / (b - 2.0);
  for (int trial = 0; trial < kMaxTrials; ++trial) {
    const double U = rng.uniform() - 0.5;
    const double V = rng.uniform();
    const double us = 0.5 - fabs(U);
    const double kf = floor((2.0 * a / us + b) * U + lam + 0.43);
    if (us >= 0.07 && V <= v_r) return (long long)kf;
    if (kf < 0.0 || (us < 0.013 && V > us)) continue;
    if (log(V) + log(inv_alpha) - log(a / (us * us) + b) <= -lam + kf * loglam - lgamma(kf + 1.0))
      return (long long)kf;
  }
  return (long long)rint(lam);
}

__global__ __launch_bounds__(256) void k_poisson_noise(const float* __restrict__ p, float* __restrict__ out,
                                                       long long* __restrict__ counts, size_t n, double photons,
                                                       double mu, unsigned long long seed, unsigned long long e0) {
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
    const double lam = photons * exp(-mu * (double)p[q]);
    const long long N = poisson_count(lam, seed, e0 + q);
    if (counts) counts[q] = N;
    out[q] = (float)(-log((double)(N > 1 ? N : 1) / photons) / mu);
  }
}

hipError_t launch_poisson_noise(const float* p, float* out, long long* counts, size_t n, double photons, double mu,
                                unsigned long long seed, unsigned long long e0, hipStream_t s) {
  const size_t blocks = std::min<size_t>(16384, (n + 255) / 256);
  hipLaunchKernelGGL(k_poisson_noise, dim3((unsigned)blocks), dim3(256), 0, s, p, out, counts, n, photons, mu, seed, e0);
  return hipGetLastError();
}

}  // namespace dc
