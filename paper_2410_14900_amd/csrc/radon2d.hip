// 2D parallel-beam Radon pair on each detector image (paper eqs. 7, 8, 11):
//
//   splat : out[k][m] = scale * sum_p w(p) img(p) Lambda(t_pk - m)     (A2d and the detector Radon)
//   interp: out(p)    = scale * w(p) sum_k lerp(rows[k], t_pk)          (A2d^T and the transposed A2d)
//
// with t_pk = i A_k + j B_k + C_k the fractional s-bin of pixel p=(i,j) on angle
// mu_k, Lambda the hat function and w the optional cosine weight D/sqrt(x^2+y^2+D^2).
// The two are exact transposes of each other for equal scales.
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "dc_internal.h"

namespace dc {

// ------------------------------------------------------------------ splat
// One workgroup owns one view and a chunk of <= kc angles whose sinogram rows
// live in LDS.  Every pixel of the view is read once per chunk.  Pixel p with
// fractional bin t = m + f deposits x(1-f) on bin m and x f on bin m+1, i.e.
//     R(m) = a(m) - b(m) + b(m-1),   a(m) = sum_{m_p = m} x_p,  b(m) = sum_{m_p = m} x_p f_p,
// so both sums land on the SAME index m_p.  They are accumulated as fixed-point
// integers packed into one 64-bit word (a + 2^32 b) with a single LDS integer
// atomic per pixel-angle (float LDS atomics are ~30x slower on this GPU, integer
// ones run at full LDS rate).  Integer addition is associative, so the result is
// bit-reproducible.  The fixed-point scale is per view: a small reduction kernel
// writes max|x| over each view to the plan's scratch, and the quantum is sized so
// that no bin's a-sum can leave 32 bits (the plan bounds how many pixels share
// a bin on one angle).
//
// The fractional bin t reaches ~n_s, where a float32 ulp is 1e-4 bin; it is kept
// in exact 32.32 fixed point instead (see the walk below).
__global__ void k_zero_u32(unsigned* __restrict__ p, int n) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) p[q] = 0u;
}

hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u32, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// max |w x| over each view, as float bits (non-negative floats order like their bits),
// into vmax[v - v0] (zeroed before)
// four consecutive storage values as float32 (one 16- or 8-byte load)
__device__ __forceinline__ void load4(const float* p, float x[4]) {
  const float4 q = *reinterpret_cast<const float4*>(p);
  x[0] = q.x; x[1] = q.y; x[2] = q.z; x[3] = q.w;
}
template <typename T>
__device__ __forceinline__ void load4(const T* p, float x[4]) {
  const uint2 q = *reinterpret_cast<const uint2*>(p);
  T h[4];
  __builtin_memcpy(h, &q, sizeof(q));
#pragma unroll
  for (int k = 0; k < 4; ++k) x[k] = to_f32(h[k]);
}

// VEC: nu is a multiple of 4, so every row starts 16-byte (float) or 8-byte
// (16-bit storage) aligned in the 16-byte aligned array, and a thread takes four
// consecutive pixels of a row with one load
template <typename Tin, bool WCOS, bool VEC>
__global__ __launch_bounds__(256) void k_view_absmax(const Tin* __restrict__ img, unsigned* __restrict__ vmax, KGrid g,
                                                     const float4* __restrict__ viewf, int v0) {
  __shared__ float red[256];
  const int v = v0 + blockIdx.y;
  const int npix = g.nu * g.nv;
  const Tin* im = img + (size_t)v * npix;
  const float D = viewf[v].x;
  float mx = 0.f;
  // whole rows per workgroup (rows blockIdx.x, + gridDim.x, ...): coalesced loads
  // and the pixel's row known without a division
  for (int j = blockIdx.x; j < g.nv; j += gridDim.x) {
    const Tin* row = im + (size_t)j * g.nu;
    const float yv = (j - g.cv) * g.dv;
    const float r2 = fmaf(yv, yv, D * D);
    // hardware rsqrt: the argument is at least D^2, far from the denormal range
    // that rsqrtf's scaling guards; the same weight as the splat's, bit for bit
    auto weigh = [&](float x, int i) {
      if (WCOS) {
        const float xu = (i - g.cu) * g.du;
        x *= D * __builtin_amdgcn_rsqf(fmaf(xu, xu, r2));
      }
      return fabsf(x);
    };
    if (VEC) {
      for (int i = 4 * threadIdx.x; i < g.nu; i += 4 * blockDim.x) {
        float x[4];
        load4(row + i, x);
#pragma unroll
        for (int k = 0; k < 4; ++k) mx = fmaxf(mx, weigh(x[k], i + k));
      }
    } else {
      for (int i = threadIdx.x; i < g.nu; i += blockDim.x) mx = fmaxf(mx, weigh(to_f32(row[i]), i));
    }
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(vmax + blockIdx.y, __float_as_uint(red[0]));   // word of view v0 + y
}

static constexpr int kSplatKC = 8;   // max angles per workgroup (registers hold one t per angle)
static constexpr int kSplatPre = 8;   // pixels loaded ahead along a line
static constexpr float kRoundMagic = 12582912.0f;       // 1.5 * 2^23
static constexpr unsigned kRoundMagicBits = 0x4B400000u;  // its bit pattern

template <typename Tin, typename Tout, bool WCOS, bool CHECKED>
__global__ __launch_bounds__(512) void k_splat(const Tin* __restrict__ img, Tout* __restrict__ out, KGrid g,
                                               const int4* __restrict__ chunks,
                                               const double* __restrict__ angd,
                                               const float4* __restrict__ viewf, float scale, int v0, int nv,
                                               int n_chunks, float qmax, const unsigned* __restrict__ vmax_bits) {
  extern __shared__ unsigned long long acc[];   // [kn][n_s + 1], index m + 1
  __shared__ double sA[16], sB[16], sC[16];
  __shared__ long long sStep[16];
  // XCD-aware order: workgroup b runs on XCD b % 8; all angle chunks of a view
  // go to the same XCD, so the view's image is fetched from HBM into one L2.
  const int xcd = blockIdx.x & 7, kb = blockIdx.x >> 3;
  const int vl = xcd + 8 * (kb / n_chunks);
  if (vl >= nv) return;
  const int4 ch = chunks[kb % n_chunks];
  const int v = v0 + vl;
  const int k0 = ch.x, kn = ch.y, colmajor = ch.z;
  const int ns = g.n_s, row = ns + 1;
  const int npix = g.nu * g.nv;
  const Tin* im = img + (size_t)v * npix;
  const float D = viewf[v].x;
  for (int q = threadIdx.x; q < kn * row; q += blockDim.x) acc[q] = 0ull;
  if (threadIdx.x < kn) {
    const int k = k0 + threadIdx.x;
    sA[threadIdx.x] = angd[3 * k];
    sB[threadIdx.x] = angd[3 * k + 1];
    sC[threadIdx.x] = angd[3 * k + 2];
    // step of t along the walk direction in 32.32 fixed point
    sStep[threadIdx.x] = (long long)llrint((colmajor ? angd[3 * k] : angd[3 * k + 1]) * 4294967296.0);
  }
  __syncthreads();
  const float vmax = __uint_as_float(vmax_bits[vl]);   // the view's word, indexed from v0
  // quantum: the largest term takes qmax units (fixed_point_qmax of the plan's
  // bound on pixels per bin), so |a| per bin stays in 31 bits and every term
  // below 2^21, where the rounding below is exact
  const float S = vmax > 0.f ? qmax / vmax : 0.f;
  // Threads own whole lines of pixels (columns when the angles spread rows,
  // rows otherwise) and walk them; t advances by an exact fixed-point step, so
  // the bin index is the high word and the fraction the low word, with a
  // rounding drift below 2^-33 bin per step.  The high word also carries the
  // angle's LDS row offset (kk * row + 1), so it is the accumulator index itself.
  const int n_lines = colmajor ? g.nv : g.nu;
  const int n_steps = colmajor ? g.nu : g.nv;
  // The lanes of a wave take every other line (waves pair up over 128 lines):
  // neighbouring lines are less than one bin apart on these angles, so adjacent
  // lanes would often add to the same word in one instruction; two lines apart they
  // do not, at the price of some 4-way bank conflicts (measured 13% faster than
  // consecutive lines, stride 4 is slower again).
  const int lane_line = ((threadIdx.x >> 7) << 7) + ((threadIdx.x & 63) << 1) + ((threadIdx.x >> 6) & 1);
  // Full chunks (kSplatKC angles, nearly all of them) run a copy of the walk
  // without the per-angle range checks.  Each walk direction (COL: lines are rows)
  // has its own copy, so the line's part of the cosine weight is computed once per
  // line (7.5 -> 6.6 VALU per pixel-angle, 1% faster).
  auto walk = [&](auto full, auto col) {
    constexpr bool FULL = decltype(full)::value;
    constexpr bool COL = decltype(col)::value;
    for (int line = lane_line; line < n_lines; line += blockDim.x) {
      long long t[kSplatKC];
  #pragma unroll
      for (int kk = 0; kk < kSplatKC; ++kk) {
        if (FULL || kk < kn) {
          const double t0 = COL ? fma((double)line, sB[kk], sC[kk]) : fma((double)line, sA[kk], sC[kk]);
          const double fl = floor(t0);
          t[kk] = ((long long)((int)fl + kk * row + 1) << 32) + (long long)(unsigned)((t0 - fl) * 4294967296.0);
        } else {
          t[kk] = 0;
        }
      }
      // the next kSplatPre pixels of the line are loaded while the current ones
      // are deposited, so each wave keeps several loads in flight
      const Tin* base = COL ? im + (size_t)line * g.nu : im + line;
      const int pitch = COL ? 1 : g.nu;
      Tin xb[kSplatPre];   // raw storage values, converted at use
  #pragma unroll
      for (int q = 0; q < kSplatPre; ++q) xb[q] = q < n_steps ? base[(size_t)q * pitch] : Tin{};
      for (int p0 = 0; p0 < n_steps; p0 += kSplatPre) {
        Tin xc[kSplatPre];
  #pragma unroll
        for (int q = 0; q < kSplatPre; ++q) xc[q] = xb[q];
        if (p0 + kSplatPre < n_steps) {
  #pragma unroll
          for (int q = 0; q < kSplatPre; ++q) {
            const int pn = p0 + kSplatPre + q;
            xb[q] = pn < n_steps ? base[(size_t)pn * pitch] : Tin{};
          }
        }
  #pragma unroll
        for (int q = 0; q < kSplatPre; ++q) {
          const int p = p0 + q;
          if (p >= n_steps) break;
          const int i = COL ? p : line, j = COL ? line : p;
          float x = to_f32(xc[q]);
          if (WCOS) {
            const float xu = (i - g.cu) * g.du, yv = (j - g.cv) * g.dv;
            x *= D * __builtin_amdgcn_rsqf(fmaf(xu, xu, fmaf(yv, yv, D * D)));
          }
          const float xs = x * S;
          // Integer rounding without conversion instructions: adding 1.5 * 2^23
          // leaves round-to-nearest-even(v) in the low mantissa bits for |v| < 2^22.
          const int qa = (int)(__float_as_uint(xs + kRoundMagic) - kRoundMagicBits);
          // high word = qb + sign extension of qa, taken from the same trick
          const unsigned hbias = kRoundMagicBits - (unsigned)(qa >> 31);
          const float xs2 = xs * 2.3283064365386963e-10f;  // xs * 2^-32
  #pragma unroll
          for (int kk = 0; kk < kSplatKC; ++kk) {
            if (FULL || kk < kn) {
              const unsigned idx = (unsigned)(t[kk] >> 32);  // kk * row + m + 1
              const unsigned lo = (unsigned)t[kk];
              const unsigned hi = __float_as_uint(fmaf(xs2, (float)lo, kRoundMagic)) - hbias;
              const unsigned long long word = ((unsigned long long)hi << 32) | (unsigned long long)(unsigned)qa;
              if (!CHECKED || idx - (unsigned)(kk * row) <= (unsigned)ns) atomicAdd(acc + idx, word);
              t[kk] += sStep[kk];
            }
          }
        }
      }
    }
  };
  if (kn == kSplatKC) {
    if (colmajor) walk(std::true_type{}, std::true_type{});
    else walk(std::true_type{}, std::false_type{});
  } else {
    if (colmajor) walk(std::false_type{}, std::true_type{});
    else walk(std::false_type{}, std::false_type{});
  }
  __syncthreads();
  // decode: word = a + 2^32 b with |a| < 2^31
  Tout* o = out + ((size_t)v * g.n_theta + k0) * ns;
  const double inv = S > 0.f ? (double)scale / (double)S : 0.0;
  for (int q = threadIdx.x; q < kn * ns; q += blockDim.x) {
    const int kk = q / ns, m = q - kk * ns;
    const long long w = (long long)acc[kk * row + m + 1];
    const long long a = (long long)(int)(unsigned)(w & 0xffffffffll);
    const long long b = (w - a) >> 32;
    const long long wp = (long long)acc[kk * row + m];
    const long long ap = (long long)(int)(unsigned)(wp & 0xffffffffll);
    const long long bp = (wp - ap) >> 32;
    o[q] = from_f32<Tout>((float)((double)(a - b + bp) * inv));
  }
}

// ----------------------------------------------------------------- interp
// One workgroup owns a 64 x 64 pixel tile of one view (512 threads, 8 pixels
// each, 8 rows apart: the per-angle set-up is shared by 8 taps; 8% faster than
// 32 x 64, itself 11% faster than 32 x 32: a wider tile shares each angle's
// window staging over more pixels).  Angles are processed in chunks of 32: for each angle the
// tile's s-range (plus margins) of the row is staged in LDS as one (c, s) pair per
// bin interval e, the line through its two samples written about the window's
// centre wc: value(th) = c + s th with th = t - 0.5 - wc measured from that centre.
// A linear-interpolation tap is then one 8-byte LDS read and one FMA on th itself
// (no fraction to form).  The form cancels at most |th| <= wl/2 times the slope's
// rounding: 3.2e-6 relative against the float64 oracle on the benchmark grid
// (2.7e-6 with 32 x 64 tiles, 1.6e-6 with 32 x 32).  Tile-local positions are
// derived from float64 per-(tile, angle) offsets, which keeps them below ~95
// bins and their float32 rounding below 6e-6 bins.
// LOCAL: windows wider than kInterpLocalAbove intervals (bins much finer than
// pixels) keep each pixel's position t - w0 in exact 32.32 fixed point, set up
// in float64 per (pixel, angle) and advanced by an exact step over the thread's
// 8 rows, and store (left sample, slope) per interval: a tap is the interval
// index (high word), its fraction (low word, 23 bits as a float in [0, 1)) and
// one FMA.  In the float form the position is a float32 of magnitude up to
// wl/2 whose rounding (and that of A, B in float32) grows with the window: at
// bins a fifth of the pixel pitch (wl = 450) it leaves 1.2e-5 against the
// oracle, above the float32 bar.
// Tile: TX x 64 pixels (TX = 32 or 64, the plan's knob; TX 8 threads); angles
// per chunk kc <= kInterpMaxKC (knob, at run time).
static constexpr int kTY = 64;
static constexpr int kTPX = kTY / 8;   // pixels per thread (rows 8 apart)

template <typename Tin, typename Tout, bool WCOS, bool LOCAL, int TX>
__global__ __launch_bounds__(TX * 8) void k_interp(const Tin* __restrict__ rows, Tout* __restrict__ out, KGrid g,
                                                   const double* __restrict__ angd,
                                                   const float4* __restrict__ viewf, float scale, int v0, int nv,
                                                   int wl, int kc, int tiles_u, int n_tiles) {
  extern __shared__ float2 win[];
  __shared__ float4 sPar[kInterpMaxKC];   // A, B, t(tile origin) - w0 - 0.5 - wc, kk * wl + wc - bits(1.5 2^23) (int bits)
  __shared__ int sW0[kInterpMaxKC];       // first bin of each angle's window
  __shared__ double sParD[LOCAL ? kInterpMaxKC : 1][3];     // LOCAL: A, B, t(tile origin) - w0 in float64
  __shared__ long long sStep8[LOCAL ? kInterpMaxKC : 1];    // LOCAL: 8 B in 32.32 fixed point
  // XCD-aware order: all tiles of a view run on one XCD (its sinogram stays in one L2)
  const int xcd = blockIdx.x & 7, kb = blockIdx.x >> 3;
  const int vl = xcd + 8 * (kb / n_tiles);
  if (vl >= nv) return;
  const int v = v0 + vl;
  const int tile = kb % n_tiles;
  const int tu = tile % tiles_u, tv = tile / tiles_u;
  const int i0 = tu * TX, j0 = tv * kTY;
  const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;  // ty in [0, 8)
  const int ns = g.n_s;
  const Tin* rv = rows + (size_t)v * g.n_theta * ns;
  float acc[kTPX];
#pragma unroll
  for (int h = 0; h < kTPX; ++h) acc[h] = 0.f;
  for (int k0 = 0; k0 < g.n_theta; k0 += kc) {
    // uniform: held in a scalar register, so the angle loop costs no vector instructions
    const int kn = __builtin_amdgcn_readfirstlane(min(kc, g.n_theta - k0));
    if (threadIdx.x < kn) {
      const int k = k0 + threadIdx.x;
      const double A = angd[3 * k], B = angd[3 * k + 1], C = angd[3 * k + 2];
      const double t00 = C + i0 * A + j0 * B;
      const double tmin = t00 + fmin(0.0, (TX - 1) * A) + fmin(0.0, (kTY - 1) * B);
      const int w0 = (int)floor(tmin) - 1;
      sW0[threadIdx.x] = w0;
      sPar[threadIdx.x] = make_float4((float)A, (float)B, (float)(t00 - w0 - 0.5 - (wl >> 1)),
                                      __int_as_float((int)((unsigned)(threadIdx.x * wl + (wl >> 1)) - kRoundMagicBits)));
      if (LOCAL) {
        sParD[threadIdx.x][0] = A;
        sParD[threadIdx.x][1] = B;
        sParD[threadIdx.x][2] = t00 - w0;
        sStep8[threadIdx.x] = (long long)llrint(8.0 * B * 4294967296.0);
      }
    }
    __syncthreads();
    // entry q = (kk, e) with q = kk wl + e; a thread's entries lie blockDim.x apart, so
    // (kk, e) advances by (blockDim.x / wl, blockDim.x % wl) with one carry, not a division
    const int dkk = blockDim.x / wl, de = blockDim.x - dkk * wl;
    int kk = threadIdx.x / wl, e = threadIdx.x - kk * wl;
    for (int q = threadIdx.x; q < kn * wl; q += blockDim.x) {
      const int m = sW0[kk] + e;
      const Tin* r = rv + (size_t)(k0 + kk) * ns;
      const float a = ((unsigned)m < (unsigned)ns) ? to_f32(r[m]) : 0.f;
      const float b = ((unsigned)(m + 1) < (unsigned)ns) ? to_f32(r[m + 1]) : 0.f;
      // float form: midpoint (a + b) / 2 at th = e - wc, slope b - a, moved to the
      // window centre; LOCAL: left sample and slope
      win[q] = LOCAL ? make_float2(a, b - a)
                     : make_float2(0.5f * (a + b) - (float)(e - (wl >> 1)) * (b - a), b - a);
      kk += dkk;
      e += de;
      if (e >= wl) {
        e -= wl;
        ++kk;
      }
    }
    __syncthreads();
    const float fx = (float)tx, fy = (float)ty;
    if constexpr (LOCAL) {
      for (int kk = 0; kk < kn; ++kk) {
        // t - w0 >= 1 for every pixel of the tile (w0 is one below the tile's lowest bin)
        const double ud = fma((double)tx, sParD[kk][0], fma((double)ty, sParD[kk][1], sParD[kk][2]));
        const double fl = floor(ud);
        long long u = ((long long)((int)fl + kk * wl) << 32) | (long long)(unsigned)((ud - fl) * 4294967296.0);
        const long long step = sStep8[kk];
#pragma unroll
        for (int h = 0; h < kTPX; ++h) {
          const unsigned lo = (unsigned)u;
          const float fr = __uint_as_float((lo >> 9) | 0x3f800000u) - 1.0f;   // fraction, 23 bits
          const float2 pr = win[(int)(u >> 32)];
          acc[h] += fmaf(fr, pr.y, pr.x);
          u += step;
        }
      }
      __syncthreads();
      continue;
    }
    for (int kk = 0; kk < kn; ++kk) {
      const float4 P = sPar[kk];
      // th = t - 0.5 relative to the window centre; rounding it to the nearest
      // integer with the 1.5 * 2^23 trick gives the interval floor(t) (an exact
      // integer t may round one lower, where both intervals give the same value)
      const float th0 = fmaf(fx, P.x, fmaf(fy, P.y, P.z));
      const float b8 = 8.f * P.y;
      const unsigned nbias = (unsigned)__float_as_int(P.w);   // window slot = bits(th + 1.5 2^23) + nbias
#pragma unroll
      for (int h = 0; h < kTPX; ++h) {
        const float th = h == 0 ? th0 : fmaf((float)h, b8, th0);   // 0 b8 + th0 is not folded
        const float y = th + kRoundMagic;
        const float2 pr = win[__float_as_uint(y) + nbias];
        acc[h] += fmaf(th, pr.y, pr.x);
      }
    }
    __syncthreads();
  }
  const float D = viewf[v].x;
  const int i = i0 + tx;
  Tout* o = out + (size_t)v * g.nu * g.nv;
#pragma unroll
  for (int h = 0; h < kTPX; ++h) {
    const int j = j0 + ty + 8 * h;
    if (i < g.nu && j < g.nv) {
      float val = scale * acc[h];
      if (WCOS) {
        float xu = (i - g.cu) * g.du, yv = (j - g.cv) * g.dv;
        val *= D * __builtin_amdgcn_rsqf(fmaf(xu, xu, fmaf(yv, yv, D * D)));
      }
      o[j * g.nu + i] = from_f32<Tout>(val);
    }
  }
}

// --------------------------------------------------------------- dispatch

// Scratch of the allocation-free splat entry point (dc_weight_radon_noalloc): one
// word per view of a call, in a static device array.  Each GPU holds its own copy
// until the process ends; host code reaches it only through the per-device
// address from hipGetSymbolAddress (the array's name is a host-side stand-in).
static __device__ __align__(256) unsigned scratch[kNoAllocViews];

static std::mutex g_scratch_mu;
static unsigned* g_scratch_ptr[kMaxDevices] = {};

hipError_t static_scratch(int device, unsigned** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    // called with `device` current (plan creation, or a call on that device's plan)
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<unsigned*>(ptr);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

hipError_t launch_splat(const Plan& p, const void* img, dc_dtype t_in, bool wcos, float scale, void* out,
                        dc_dtype t_out, int v0, int nv, hipStream_t s, unsigned* vmax_words) {
  const size_t lds = (size_t)p.splat_kc * (p.kg.n_s + 1) * sizeof(unsigned long long);
  dim3 grid(8 * ((nv + 7) / 8) * p.n_chunks);
  // one max word per view of the call: the plan's scratch, or the caller's (the static array)
  unsigned* vmax = vmax_words ? vmax_words : p.d_scratch + v0;
  hipError_t e = launch_zero_u32(vmax, nv, s);
  if (e != hipSuccess) return e;
  return by_dtype(t_in, [&](auto tin) {
    using Tin = decltype(tin);
    const int mblocks = std::max(1, std::min(64, p.kg.nv / 8));   // about 8 rows per workgroup
#define DC_ABSMAX(W, VEC)                                                                                    \
  hipLaunchKernelGGL((k_view_absmax<Tin, W, VEC>), dim3(mblocks, nv), dim3(256), 0, s, (const Tin*)img, vmax, \
                     p.kg, (const float4*)p.d_view, v0)
    const bool vec = p.kg.nu % 4 == 0;
    if (wcos) {
      if (vec) DC_ABSMAX(true, true); else DC_ABSMAX(true, false);
    } else {
      if (vec) DC_ABSMAX(false, true); else DC_ABSMAX(false, false);
    }
#undef DC_ABSMAX
    hipError_t e2 = hipGetLastError();
    if (e2 != hipSuccess) return e2;
    return by_dtype(t_out, [&](auto tout) {
      using Tout = decltype(tout);
#define DC_SPLAT(W, C)                                                                                         \
  hipLaunchKernelGGL((k_splat<Tin, Tout, W, C>), grid, dim3(512), lds, s, (const Tin*)img, (Tout*)out, p.kg,  \
                     p.d_chunks, p.d_ang, (const float4*)p.d_view, scale, v0, nv, p.n_chunks, p.splat_qmax, \
                     vmax)
      if (wcos) {
        if (p.splat_checked) DC_SPLAT(true, true); else DC_SPLAT(true, false);
      } else {
        if (p.splat_checked) DC_SPLAT(false, true); else DC_SPLAT(false, false);
      }
#undef DC_SPLAT
      return hipGetLastError();
    });
  });
}

hipError_t launch_interp(const Plan& p, const void* rows, dc_dtype t_in, bool wcos, float scale, void* out,
                         dc_dtype t_out, int v0, int nv, hipStream_t s) {
  const int TXr = p.shape.interp_tx, kc = p.shape.interp_kc;
  const int tiles_u = (p.kg.nu + TXr - 1) / TXr, tiles_v = (p.kg.nv + kTY - 1) / kTY;
  const size_t lds = (size_t)kc * p.interp_wl * sizeof(float2);
  const int n_tiles = tiles_u * tiles_v;
  dim3 grid(8 * ((nv + 7) / 8) * n_tiles);
  return by_dtype(t_in, [&](auto tin) {
    using Tin = decltype(tin);
    return by_dtype(t_out, [&](auto tout) {
      using Tout = decltype(tout);
#define DC_INTERP1(W, L, TX)                                                                                     \
  hipLaunchKernelGGL((k_interp<Tin, Tout, W, L, TX>), grid, dim3(TX * 8), lds, s, (const Tin*)rows, (Tout*)out,  \
                     p.kg, p.d_ang, (const float4*)p.d_view, scale, v0, nv, p.interp_wl, kc, tiles_u, n_tiles)
#define DC_INTERP(W, L)                      \
  do {                                       \
    if (TXr == 32) DC_INTERP1(W, L, 32);     \
    else DC_INTERP1(W, L, 64);               \
  } while (0)
      const bool local = p.interp_wl > kInterpLocalAbove;
      if (wcos) {
        if (local) DC_INTERP(true, true); else DC_INTERP(true, false);
      } else {
        if (local) DC_INTERP(false, true); else DC_INTERP(false, false);
      }
#undef DC_INTERP
#undef DC_INTERP1
      return hipGetLastError();
    });
  });
}

}  // namespace dc
