// Cone-beam backprojection (paper eq. 5 with the detector weight of eq. 11 folded
// in) and its exact transpose, the cone-beam forward projection:
//
//   f(x)       (+)= sum_v (D/U)^2 sum_{i,j} gF_v[j][i] Lambda(i* - i) Lambda(j* - j)
//   GgF_v[j][i]  = sum_x (D/U)^2 Gf(x)    Lambda(i* - i) Lambda(j* - j)
//
// with the per-view projective map i* = num_u/den, j* = num_v/den, den = U/D,
// all affine in the voxel index (float64 table built by the plan).
//
// Backprojection work mapping: a workgroup owns a 16 x 32 x 8 voxel block and a
// thread one (x, y) column segment of 8 voxels, walked in z (8 rather than 16
// keeps the kernel at 3 waves per SIMD; measured 4% faster); lanes of a wave
// cover 16 consecutive x of 4 rows, so volume writes are 64-byte segments.  Per view, the block's
// detector footprint is staged in LDS (converted to float32 from the storage
// type) and the taps are LDS reads; the next view's footprint is fetched into
// registers while the current one is interpolated (double buffering, one barrier
// per view).  For every view the thread forms its column's projection
// coefficients in float64 relative to an integer detector origin near the
// column's projection, so the float32 per-voxel coordinates stay small and
// their rounding far below 1e-5 pixel.
#include <algorithm>
#include <type_traits>

#include "dc_internal.h"

namespace dc {

// Block: kBX x BY x kZC voxels, BY = 16 or 32 (the plan's knob), kBX BY threads.
static constexpr int kBX = 16, kZC = 8;
// kernel template value for a launch over samples of different forms (ConeForm)
static constexpr int kConeMixed = 3;

static constexpr float kRoundMagic = 12582912.0f;         // 1.5 * 2^23
static constexpr unsigned kRoundMagicBits = 0x4B400000u;  // its bit pattern

// Two terms a and b rounded with the 1.5 * 2^23 trick (|a|, |b| < 2^22), as the
// 64-bit word b 2^32 + a: subtracting both biases at once lets the borrow carry
// the sign of a into the high word.
__device__ __forceinline__ unsigned long long pack_terms(float a_biased, float b_biased) {
  constexpr unsigned long long kBias = ((unsigned long long)kRoundMagicBits << 32) | kRoundMagicBits;
  return ((((unsigned long long)__float_as_uint(b_biased)) << 32) | __float_as_uint(a_biased)) - kBias;
}

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
  // iu0, jv0 only anchor the float offsets below (formed exactly in float64), so
  // any integer within a pixel of the projection serves: the hardware reciprocal does
  const float rden = __builtin_amdgcn_rcpf((float)den);
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

// Column set-up when neither den nor num_u has a z-term (the detector's v axis
// is parallel to z, as on circular orbits): the column keeps one u, so its tap
// column i, the fraction fu and the weight (D/U)^2 hold for the whole segment,
// and only v moves along z.
struct ColumnMapZ {
  float r2, fu;     // (D/U)^2 and the fraction of u in its cell
  float w0m, dw;    // v - jv0 - 1/2 at the segment start and its z step
  int i, jv0;       // detector column of the left taps, anchor row of v
};

__device__ __forceinline__ ColumnMapZ column_map_z(const double* __restrict__ P, int ix, int iy, int iz0) {
  const double den = fma((double)ix, P[0], fma((double)iy, P[1], P[3]));
  const double nu = fma((double)ix, P[4], fma((double)iy, P[5], P[7]));
  const double nv = fma((double)ix, P[8], fma((double)iy, P[9], fma((double)iz0, P[10], P[11])));
  const float rden = __builtin_amdgcn_rcpf((float)den);
  const int iu0 = (int)floorf((float)nu * rden), jv0 = (int)floorf((float)nv * rden);
  const float u = (float)fma(-(double)iu0, den, nu) * rden;
  const float yu = (u - 0.5f) + kRoundMagic;
  ColumnMapZ c;
  c.fu = u - (yu - kRoundMagic);
  c.i = iu0 + (int)(__float_as_uint(yu) - kRoundMagicBits);
  c.jv0 = jv0;
  c.r2 = rden * rden;
  c.w0m = (float)fma(-(double)jv0, den, nv) * rden - 0.5f;
  c.dw = (float)P[10] * rden;
  return c;
}

// Column set-up of the cone adjoint's general forms.  The numerators are taken
// about iu0 + 1/2 and jv0 + 1/2 (any integers within a pixel of the projection:
// the hardware reciprocal serves), so n rr = u - iu0 - 1/2 and likewise v, and
// every coordinate is scaled by sf = 1/sqrt(S), so rr^2 = S (D/U)^2 carries the
// fixed-point quantum.  den and the numerators at the segment start are formed in
// float64 (where they cancel).  With FLOAT_STEPS (den changes by at most 5e-4
// of itself per voxel step) their z-steps are formed in float from the view's
// scaled steps zd, zu, zv (dden, dnum_u, dnum_v): the product au zd is then at
// most 5e-4 au den, so the step's error stays near one rounding of it;
// otherwise they are formed in float64.
struct ColumnMapF {
  float den, lu, lv;   // at the first voxel of the segment
  float ldu, ldv;      // z-steps of the numerators
  int iu0, jv0;
};

template <bool FLOAT_STEPS>
__device__ __forceinline__ ColumnMapF column_map_fp(const double* __restrict__ P, int ix, int iy, int iz0, float sf,
                                                    float zd, float zu, float zv) {
  const double den = fma((double)ix, P[0], fma((double)iy, P[1], fma((double)iz0, P[2], P[3])));
  const double nu = fma((double)ix, P[4], fma((double)iy, P[5], fma((double)iz0, P[6], P[7])));
  const double nv = fma((double)ix, P[8], fma((double)iy, P[9], fma((double)iz0, P[10], P[11])));
  const float rden = __builtin_amdgcn_rcpf((float)den);
  const float yu = fmaf((float)nu, rden, kRoundMagic), yv = fmaf((float)nv, rden, kRoundMagic);
  const float au = (yu - kRoundMagic) + 0.5f, av = (yv - kRoundMagic) + 0.5f;   // exact
  ColumnMapF c;
  c.iu0 = (int)(__float_as_uint(yu) - kRoundMagicBits);
  c.jv0 = (int)(__float_as_uint(yv) - kRoundMagicBits);
  c.den = (float)den * sf;
  c.lu = (float)fma(-(double)au, den, nu) * sf;
  c.lv = (float)fma(-(double)av, den, nv) * sf;
  if (FLOAT_STEPS) {
    c.ldu = fmaf(-au, zd, zu);
    c.ldv = fmaf(-av, zd, zv);
  } else {
    c.ldu = (float)fma(-(double)au, P[2], P[6]) * sf;
    c.ldv = (float)fma(-(double)av, P[2], P[10]) * sf;
  }
  return c;
}

static constexpr int kBufferWord3 = 0x00020000;   // raw buffer resource word 3 on this GPU family

// raw buffer load of one storage element (offsets past the resource read 0)
__device__ __forceinline__ void buffer_load_raw(__amdgpu_buffer_rsrc_t r, unsigned off, float& x) {
  x = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ __forceinline__ void buffer_load_raw(__amdgpu_buffer_rsrc_t r, unsigned off, bf16_t& x) {
  x.bits = __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
}
__device__ __forceinline__ void buffer_load_raw(__amdgpu_buffer_rsrc_t r, unsigned off, _Float16& x) {
  x = __builtin_bit_cast(_Float16, (unsigned short)__builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0));
}

template <typename T>
__device__ __forceinline__ float tap(const T* __restrict__ img, int i, int j, int nu, int nv) {
  return ((unsigned)i < (unsigned)nu && (unsigned)j < (unsigned)nv) ? to_f32(img[j * nu + i]) : 0.f;
}

// Footprint of a voxel block on view v: the projective image of the index box
// lies in the convex hull of its 8 projected corners, so [floor(min)-1,
// floor(max)+2] in each detector direction covers every bilinear tap (with a
// pixel of margin for rounding).  Computed by lanes 0..7 of every wave and
// combined with shuffles, so each wave knows the box without a barrier.
struct Box {
  int i_lo, j_lo, w, h;
};

__device__ __forceinline__ Box block_footprint(const double* __restrict__ P, int bx0, int bx1, int by0, int by1,
                                               int bz0, int bz1) {
  const int lane = threadIdx.x & 63;
  const int c = lane & 7;
  const double x = (c & 1) ? bx1 : bx0, y = (c & 2) ? by1 : by0, z = (c & 4) ? bz1 : bz0;
  const double den = fma(x, P[0], fma(y, P[1], fma(z, P[2], P[3])));
  const double nu = fma(x, P[4], fma(y, P[5], fma(z, P[6], P[7])));
  const double nv = fma(x, P[8], fma(y, P[9], fma(z, P[10], P[11])));
  // a float reciprocal is ample here: its error (~1e-4 pixel) is far inside the box margin
  const float rd = __builtin_amdgcn_rcpf((float)den);
  float iu = (float)nu * rd, jv = (float)nv * rd;
  float imin = iu, imax = iu, jmin = jv, jmax = jv;
#pragma unroll
  for (int m = 1; m < 8; m <<= 1) {
    imin = fminf(imin, __shfl_xor(imin, m, 8));
    imax = fmaxf(imax, __shfl_xor(imax, m, 8));
    jmin = fminf(jmin, __shfl_xor(jmin, m, 8));
    jmax = fmaxf(jmax, __shfl_xor(jmax, m, 8));
  }
  imin = fmaxf(__shfl(imin, 0), -1.0e6f);
  imax = fminf(__shfl(imax, 0), 1.0e6f);
  jmin = fmaxf(__shfl(jmin, 0), -1.0e6f);
  jmax = fminf(__shfl(jmax, 0), 1.0e6f);
  Box b;
  b.i_lo = (int)floorf(imin) - 1;
  b.j_lo = (int)floorf(jmin) - 1;
  b.w = (int)floorf(imax) + 3 - b.i_lo;
  b.h = (int)floorf(jmax) + 3 - b.j_lo;
  return b;
}

// Staging classes and forms whose kernel is compiled for 6 waves per SIMD (three
// 512-thread workgroups per CU): the quadratic and reciprocal forms with 4 or 8
// staged rows per thread, the classes real geometries use (80 registers, a few
// spilled; 7% faster on C2 than at 4 waves).  The others keep the default.
template <int STAGE, int FORM>
inline constexpr bool kBpSixWaves = (FORM == kConeQuadratic || FORM == kConeGeneral) && STAGE > 0 && STAGE <= 8;

// STAGE = staged footprint rows per thread and view and PITCH = pixels between
// staged rows (64 or 128): the plan picks the smallest pitch that holds the widest
// footprint and the smallest STAGE whose STAGE x (threads / PITCH) rows hold the
// tallest.  STAGE == 0 selects direct global taps.  FORM
// (staged form only) is the plan's choice for the sample (ConeForm), or
// kConeMixed: a launch over samples of different forms reads each workgroup's
// form from `forms` (one entry per sample).
template <typename T, int STAGE, int PITCH, int FORM, int BY>
__global__ __launch_bounds__(kBX * BY) __attribute__((amdgpu_waves_per_eu(kBpSixWaves<STAGE, FORM> ? 6 : 1)))
void k_cone_bp(const T* __restrict__ gF, float* __restrict__ f, KGrid g,
                                                 const double* __restrict__ proj, int acc_in, int relu, int v0,
                                                 int nv, const int* __restrict__ first, int s_lo, int nzb,
                                                 const int* __restrict__ forms) {
  constexpr int kBPThreads = kBX * BY;
  // staged rows lie kLP floats apart in LDS: 8 past the row's pixels, so a pixel and the
  // one below it fall in different banks (with rows exactly 64 or 128 floats apart they
  // share one, and lanes on neighbouring rows conflicted at 2.8 cycles per read)
  constexpr int kLP = PITCH + 8;
  constexpr int kTile = STAGE > 0 ? STAGE * (kBPThreads / PITCH) * kLP : 1;
  __shared__ float tile[2][kTile];
  const int tid = threadIdx.y * kBX + threadIdx.x;
  // grid z = (sample, z-block): this workgroup sums the views of its sample that
  // lie in [v0, v0 + nv) into that sample's volume
  const int zb = blockIdx.z % nzb, smp = s_lo + blockIdx.z / nzb;
  {
    const int vb = max(v0, first[smp]), ve = min(v0 + nv, first[smp + 1]);
    v0 = vb;
    nv = max(0, ve - vb);
  }
  f += (size_t)smp * g.nx * g.ny * g.nz;
  const int bx0 = blockIdx.x * kBX, by0 = blockIdx.y * BY, bz0 = zb * kZC;
  const int bx1 = min(g.nx, bx0 + kBX) - 1, by1 = min(g.ny, by0 + BY) - 1, bz1 = min(g.nz, bz0 + kZC) - 1;
  const int ix = bx0 + threadIdx.x, iy = by0 + threadIdx.y, iz0 = bz0;
  float acc[kZC];
#pragma unroll
  for (int z = 0; z < kZC; ++z) acc[z] = 0.f;
  const size_t npix = (size_t)g.nu * g.nv;
  if constexpr (STAGE == 0) {
    for (int v = v0; v < v0 + nv; ++v) {
      const ColumnMap c = column_map(proj + 12 * v, ix, iy, iz0);
      const T* img = gF + (size_t)v * npix;
#pragma unroll
      for (int z = 0; z < kZC; ++z) {
        const float den = z == 0 ? c.den : fmaf((float)z, c.dden, c.den);
        const float r = __builtin_amdgcn_rcpf(den);
        const float u = (z == 0 ? c.lu : fmaf((float)z, c.ldu, c.lu)) * r;
        const float w = (z == 0 ? c.lv : fmaf((float)z, c.ldv, c.lv)) * r;
        const float fu0 = floorf(u), fw0 = floorf(w);
        const float fu = u - fu0, fw = w - fw0;
        const int i = c.iu0 + (int)fu0, j = c.jv0 + (int)fw0;
        const float a00 = tap(img, i, j, g.nu, g.nv), a01 = tap(img, i + 1, j, g.nu, g.nv);
        const float a10 = tap(img, i, j + 1, g.nu, g.nv), a11 = tap(img, i + 1, j + 1, g.nu, g.nv);
        const float top = fmaf(fu, a01 - a00, a00), bot = fmaf(fu, a11 - a10, a10);
        acc[z] = fmaf(r * r, fmaf(fw, bot - top, top), acc[z]);
      }
    }
  } else {
    // raw storage values: converted to float32 only when written to LDS, so
    // no use of a load comes before the interpolation of the current view
    T stg[STAGE > 0 ? STAGE : 1];
    // fetch view v's footprint into registers: staged row r of the box (detector
    // row j_lo + r) sits at tile[r * kLP + c], and PITCH / 64 whole waves stage
    // one row, kBPThreads / PITCH rows per pass, so a wave's row is uniform and
    // its address arithmetic scalar.  The loads go through a resource spanning the
    // view's image: a pixel left or right of the detector takes an offset past the
    // resource's end, and so does every pixel of a row above or below it (a
    // negative offset wraps above 2^31, past the image's bytes), which reads 0, so
    // no load sits behind a branch.  Rows and columns past the box are staged too
    // and never read.
    const unsigned img_bytes = (unsigned)(npix * sizeof(T));   // < 2^31: the plan caps nu nv at 2^31 / 4
    constexpr int kRowsPerPass = STAGE > 0 ? kBPThreads / PITCH : 1;
    const int scol = tid & (PITCH - 1);
    const int srow = __builtin_amdgcn_readfirstlane(tid / PITCH);
    auto load_stage = [&](int v, const Box& b) {
      const __amdgpu_buffer_rsrc_t im =
          __builtin_amdgcn_make_buffer_rsrc((void*)(gF + (size_t)v * npix), (short)0, (int)img_bytes, kBufferWord3);
      const int i_lo = __builtin_amdgcn_readfirstlane(b.i_lo), j_lo = __builtin_amdgcn_readfirstlane(b.j_lo);
      const bool in = (unsigned)(i_lo + scol) < (unsigned)g.nu;
      const unsigned cb = (unsigned)scol * (unsigned)sizeof(T);
#pragma unroll
      for (int s = 0; s < STAGE; ++s) {
        const int jj = j_lo + srow + s * kRowsPerPass;
        const unsigned off = (unsigned)(jj * g.nu + i_lo) * (unsigned)sizeof(T) + cb;
        buffer_load_raw(im, in ? off : img_bytes, stg[s]);
      }
    };
    // element s of thread tid is staged row srow + s kRowsPerPass, column scol.
    // Nothing reads this buffer until the barrier that ends the current view
    auto store_stage = [&](int buf) {
#pragma unroll
      for (int s = 0; s < STAGE; ++s) tile[buf][(srow + s * kRowsPerPass) * kLP + scol] = to_f32(stg[s]);
    };
    // Footprints are computed by one wave per view, two views ahead, and passed
    // on in a two-slot LDS ring: the box of view v sits in slot (v - v0) & 1 from
    // the barrier that ends iteration v - 2 until all threads have read it at the
    // start of iteration v - 1, after which the slot takes the box of view v + 2.
    __shared__ int4 sBox[2];
    const int wave = tid >> 6;
    auto publish = [&](int v, int slot) {
      const Box b = block_footprint(proj + 12 * v, bx0, bx1, by0, by1, bz0, bz1);
      if ((tid & 63) == 0) sBox[slot] = make_int4(b.i_lo, b.j_lo, b.w, b.h);
    };
    auto box_of = [&](int slot) {
      const int4 b = sBox[slot];
      return Box{b.x, b.y, b.z, b.w};
    };
    Box cur{0, 0, 0, 0};
    if (nv > 0) {
      if (wave < 2 && wave < nv) publish(v0 + wave, wave);
      __syncthreads();
      cur = box_of(0);
      load_stage(v0, cur);
      store_stage(0);
    }
    __syncthreads();
    // the view loop for one form F (kConeMixed takes the sample's form at run time:
    // one uniform branch per workgroup, the same arithmetic as the form's own kernel)
    auto view_loop = [&](auto form_tag) __attribute__((always_inline)) {
    constexpr int F = decltype(form_tag)::value;
    for (int v = v0; v < v0 + nv; ++v) {
      const int buf = (v - v0) & 1;
      Box nxt{0, 0, 0, 0};
      const bool more = v + 1 < v0 + nv;
      if (more) {
        nxt = box_of(buf ^ 1);
        load_stage(v + 1, nxt);
      }
      if (v + 2 < v0 + nv && wave == ((v - v0) & 3)) publish(v + 2, buf);
      const float* t = tile[buf];
      // Tap indices of voxels inside the volume need no clamping: every voxel of the
      // block's box [bx0, bx1] x [by0, by1] x [bz0, bz1] projects inside the convex
      // hull of its corners' projections, and the box (at most PITCH wide and
      // STAGE kRowsPerPass tall, by the plan) extends that hull by at least one
      // pixel on each side (float rounding of the corners and of the
      // per-voxel walk is below 1e-4 pixel).  Padding lanes and slices (ix > bx1,
      // iy > by1 or iz > bz1 when a volume side is not a multiple of the block)
      // form taps from points outside that box, sometimes behind the source
      // (den <= 0), so their LDS addresses can leave the tile or the workgroup's
      // LDS.  Nothing depends on those reads: LDS loads never fault (past the
      // allocation they return 0, inside it any value), and the results of those
      // lanes and slices are never written (the guards at the end).
      if constexpr (F == kConeZinv) {
        const ColumnMapZ c = column_map_z(proj + 12 * v, ix, iy, iz0);
        const float* tc = t + (c.i - cur.i_lo);
        // row index = bits(round(w - 1/2) + 1.5 * 2^23) - bias, in tile rows
        const unsigned jbias = kRoundMagicBits - (unsigned)(c.jv0 - cur.j_lo);
#pragma unroll
        for (int z = 0; z < kZC; ++z) {
          const float wm = z == 0 ? c.w0m : fmaf((float)z, c.dw, c.w0m);
          const float yw = wm + kRoundMagic;
          const float fw = (wm - (yw - kRoundMagic)) + 0.5f;
          const float* r0 = tc + (__float_as_uint(yw) - jbias) * kLP;
          const float a00 = r0[0], a01 = r0[1], a10 = r0[kLP], a11 = r0[kLP + 1];
          const float top = fmaf(c.fu, a01 - a00, a00), bot = fmaf(c.fu, a11 - a10, a10);
          acc[z] = fmaf(c.r2, fmaf(fw, bot - top, top), acc[z]);
          if ((z & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
      } else {
        // numerators about iu0 + 1/2, jv0 + 1/2: n r = u - iu0 - 1/2 (and likewise v)
        const float zd = (float)proj[12 * v + 2];
        const ColumnMapF c = column_map_fp<F == kConeQuadratic>(proj + 12 * v, ix, iy, iz0, 1.0f, zd,
                                                                (float)proj[12 * v + 6], (float)proj[12 * v + 10]);
        const int oi = c.iu0 - cur.i_lo, oj = c.jv0 - cur.j_lo;
        // kConeQuadratic (den moves by at most 5e-4 of itself per voxel step): 1/den
        // along the column is its quadratic Taylor polynomial about the column's middle
        // zc, whose remainder is below (3.5 x 5e-4)^3 of it, far below float rounding
        constexpr float zc = 0.5f * (kZC - 1);
        const float dc = F == kConeQuadratic ? fmaf(zc, zd, c.den) : c.den;
        float r0 = __builtin_amdgcn_rcpf(dc);
        r0 = fmaf(r0, fmaf(-dc, r0, 1.0f), r0);
        const float r1 = -r0 * r0 * zd, r2 = -r1 * r0 * zd;   // 1/den = r0 + r1 (z - zc) + r2 (z - zc)^2
#pragma unroll
        for (int z = 0; z < kZC; ++z) {
          const float tz = (float)z - zc;
          const float r = F == kConeQuadratic ? fmaf(tz, r1, fmaf(tz * tz, r2, r0))
                          : z == 0            ? r0
                                              : __builtin_amdgcn_rcpf(fmaf((float)z, zd, c.den));
          const float nu = z == 0 ? c.lu : fmaf((float)z, c.ldu, c.lu);
          const float nw = z == 0 ? c.lv : fmaf((float)z, c.ldv, c.lv);
          // one fused rounding with the 1.5 * 2^23 trick gives the cell floor(u) (an
          // exact integer u may give the cell below with fu = 1: the same value,
          // inside the box margin), a second fused form the fraction
          const float yu = fmaf(nu, r, kRoundMagic), yw = fmaf(nw, r, kRoundMagic);
          const float fu = fmaf(nu, r, kRoundMagic - yu) + 0.5f, fw = fmaf(nw, r, kRoundMagic - yw) + 0.5f;
          const int i = oi + (int)(__float_as_uint(yu) - kRoundMagicBits);
          const int j = oj + (int)(__float_as_uint(yw) - kRoundMagicBits);
          const int q = j * kLP + i;
          const float a00 = t[q], a01 = t[q + 1], a10 = t[q + kLP], a11 = t[q + kLP + 1];
          const float top = fmaf(fu, a01 - a00, a00), bot = fmaf(fu, a11 - a10, a10);
          acc[z] = fmaf(r * r, fmaf(fw, bot - top, top), acc[z]);
          // Finish every two voxels before the next pair's reads: an empty asm that
          // takes the accumulator as an operand keeps the compiler from sinking the
          // math below later reads (it would hoist all eight voxels' reads and hold
          // their values), so the kernel fits 80 registers and three workgroups per CU
          if ((z & 1) == 1) {
            asm volatile("" : "+v"(acc[z]));
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
      if (more) store_stage(buf ^ 1);
      __syncthreads();
      cur = nxt;
    }
    };
    if constexpr (FORM == kConeMixed) {
      const int fs = forms[smp];
      if (fs == kConeZinv) view_loop(std::integral_constant<int, kConeZinv>{});
      else if (fs == kConeQuadratic) view_loop(std::integral_constant<int, kConeQuadratic>{});
      else view_loop(std::integral_constant<int, kConeGeneral>{});
    } else {
      view_loop(std::integral_constant<int, FORM>{});
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

// ------------------------------------------------------------- transpose
// Gather form of the transpose, without global atomics: one workgroup owns one
// 20 x 64 pixel tile of kFV consecutive views and visits every voxel whose bilinear
// footprint touches it on any of them (each voxel segment is loaded once and
// projected on every view), i.e. i* in [i0-1, i1), j* in [j0-1, j1).  One view per
// workgroup is fastest at 0.5 mm voxels / 0.6 mm pixels: the frusta of neighbouring
// views differ by a few voxels at the ends of the rays, so a shared x-run is
// mostly wasted on each of them, while the segment loads it would share come
// from L2.  Wider tiles amortise the conservative ends of each x-run (72% of the
// evaluated voxel-views land in the tile at 20-24 pixels, 50% at 8 x 64 over
// 4 views).  In voxel-index space these
// are four half-spaces L_k(x) >= 0 (affine because the projection is
// projective with a positive denominator).  The voxels are enumerated as
// runs of 16-voxel z-segments along x or y (per view, across the rays): every
// (z-segment, y) row of the volume (or (z-segment, x) row) is intersected with
// the four half-spaces (a conservative interval along the run; the exact test is
// made per voxel), the non-empty rows are compacted into an LDS list, and a
// flattened index over the list gives every lane one (x, y, z-segment) item,
// walked in z like the backprojection.
//
// A voxel with fractional projection (ib + fu, jb + fv) and weight g adds
// g(1-fu)(1-fv), g fu(1-fv), g(1-fu)fv, g fu fv to its four taps.  With the
// centred fractions a = fu - 1/2 and b = fv - 1/2 (what the rounding leaves,
// so no second subtraction) the four sums A = sum g, B = sum g a, C = sum g b,
// E = sum g a b are kept at index (ib, jb) as fixed-point integers packed two
// per 64-bit word and added with LDS integer atomics; each tap weight is
// (1/2 -+ a)(1/2 -+ b), so the tile is decoded at the end as
//   out(i,j) = A/4 [c + l + d + e] + B/2 [-c + l - d + e] + C/2 [-c - l + d + e]
//              + E [c - l - d + e]
// over the cell itself (c) and its left (l), lower (d) and lower-left (e) neighbours.
// Integer sums make the result bit-reproducible.  The fixed-point quantum comes
// from max |Gf| (a reduction kernel into the plan's scratch, which also applies
// the ReLU mask once into the plan's volume buffer) and the per-view bound on
// (D/U)^2, sized so no index's sums leave 32 bits.  Only z-layers whose
// box can reach the tile's window are scanned.
// Tile: TI x kFTJ pixels, TI = 16, 20 or 24 (the plan's knob).
// kFROWS: rows per enumeration batch; 256 keeps the 20-pixel tile's LDS at 26.7 KB, so
// six workgroups share a CU (2% faster at C2 than 512 rows at five)
static constexpr int kFTJ = 64, kFZS = kConeBrick, kFROWS = 256;
static constexpr int kFH = kFTJ + 1;

__device__ __forceinline__ int block_exclusive_scan_256(int v, int* tmp) {
  // inclusive Hillis-Steele over 256 threads in LDS, returns the exclusive prefix
  const int t = threadIdx.x;
  tmp[t] = v;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {
    int add = t >= d ? tmp[t - d] : 0;
    __syncthreads();
    tmp[t] += add;
    __syncthreads();
  }
  int incl = tmp[t];
  __syncthreads();
  return incl - v;
}

// The gradient (times the ReLU mask when there is one) rewritten in z-bricks,
// [ceil(nz/16)][ny][nx][16] per sample, with zeros past the last slice, so a
// 16-voxel z-segment is 64 contiguous bytes; and max |Gf * mask| per sample, as
// float bits.  One thread per brick: the reads of a slice are coalesced along x,
// and the 64-byte brick is written at once.
__global__ __launch_bounds__(256) void k_vol_brick(const float* __restrict__ Gf, const float* __restrict__ f_relu,
                                                   int nx, int ny, int nz, unsigned* __restrict__ out,
                                                   float* __restrict__ bricks) {
  __shared__ float red[256];
  // grid y = sample: one volume of nx ny nz voxels each
  const size_t plane = (size_t)nx * ny, n = plane * nz;
  const int nzs = (nz + kFZS - 1) / kFZS;
  const size_t ncol = plane * nzs;
  Gf += (size_t)blockIdx.y * n;
  if (f_relu) f_relu += (size_t)blockIdx.y * n;
  bricks += (size_t)blockIdx.y * ncol * kFZS;
  out += blockIdx.y;
  float mx = 0.f;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < ncol; q += (size_t)gridDim.x * blockDim.x) {
    const size_t zs = q / plane, xy = q - zs * plane;
    const int nzv = min(kFZS, nz - (int)zs * kFZS);
    const size_t src = zs * kFZS * plane + xy;
    float v[kFZS];
#pragma unroll
    for (int z = 0; z < kFZS; ++z) v[z] = z < nzv ? Gf[src + z * plane] : 0.f;
    if (f_relu) {
#pragma unroll
      for (int z = 0; z < kFZS; ++z) v[z] = z < nzv && f_relu[src + z * plane] > 0.f ? v[z] : 0.f;
    }
#pragma unroll
    for (int z = 0; z < kFZS; ++z) mx = fmaxf(mx, fabsf(v[z]));
    float4* dst = reinterpret_cast<float4*>(bricks + q * kFZS);
#pragma unroll
    for (int k = 0; k < kFZS / 4; ++k) dst[k] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, __float_as_uint(red[0]));
}

static constexpr int kFMaxLayers = (1024 + kFZS - 1) / kFZS;   // z-layers of the deepest volume (nz <= 1024)

static constexpr int kFV = 1;   // consecutive views per workgroup

// S[w] for a runtime w without dynamic register indexing
__device__ __forceinline__ float pick(const float (&S)[kFV], int w) {
  float r = S[0];
#pragma unroll
  for (int k = 1; k < kFV; ++k) r = w == k ? S[k] : r;
  return r;
}


// Gf: the z-bricked (masked) gradient written by k_vol_brick.
// FORM (ConeForm) as in the backprojection; with kConeZinv each (segment, view)
// has one u, one tap column and one weight, and a segment whose column misses
// the tile is skipped whole.  With kConeQuadratic (den changes by at most 5e-4 of
// itself per voxel step) 1/den along the segment is its quadratic Taylor
// polynomial about the segment's middle: the remainder is below (7.5 x 5e-4)^3 =
// 5.3e-8 of it, float rounding, and every voxel's reciprocal is independent.
// Compiled for 6 waves per SIMD: the 16-pixel tile (26 KB of LDS) then runs six
// workgroups per CU at 80 registers (7.2 ms on C2 against 8.3 at five); the wider
// tiles' LDS holds them to five or four whatever the register count.
template <typename Tout, int FORM, int TI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 6))) void k_cone_fp(const float* __restrict__ Gf, Tout* __restrict__ GgF, KGrid g,
                                                 const double* __restrict__ proj, const float* __restrict__ rmax2,
                                                 int v0, int nv, int tiles_u, int n_tiles, float qmax,
                                                 const unsigned* __restrict__ gmax_bits,
                                                 const int* __restrict__ first, int s_lo, int s_hi, int ngroups,
                                                 const int* __restrict__ forms) {
  __shared__ double sL[kFV][4][4], sNegInvA[kFV][4];
  __shared__ int sRow[kFROWS], sXlo[kFROWS], sPre[kFROWS + 1];
  __shared__ unsigned char sLay[kFROWS];   // z-layer of each listed row (sRow holds its fixed coordinate)
  __shared__ int sScan[256];
  __shared__ int sCount, sNL;
  __shared__ unsigned char sLayerOn[kFMaxLayers];
  __shared__ int sLayer[kFMaxLayers];
  constexpr int kFTI = TI, kFW = TI + 1;
  __shared__ unsigned long long sAB[kFV][kFW * kFH], sCE[kFV][kFW * kFH];
  // XCD-aware order: workgroup b runs on XCD b % 8; each XCD takes every 8th
  // tile and sweeps it through all view groups, so the ~100 workgroups resident
  // on an XCD share one tile, whose voxels over all views (a thin annulus)
  // stay in that XCD's L2.
  const int xcd = blockIdx.x & 7, k = blockIdx.x >> 3;
  const int tile = xcd + 8 * (k / ngroups);
  if (tile >= n_tiles) return;
  // view groups of up to kFV consecutive views, restarted at every sample's first
  // view, so a group reads one sample's volume
  int grp = k % ngroups, smp = s_lo, va = v0, nvw = 0;
  for (; smp <= s_hi; ++smp) {
    const int vb = max(v0, first[smp]), ve = min(v0 + nv, first[smp + 1]);
    const int ng = (ve - vb + kFV - 1) / kFV;
    if (grp < ng) {
      va = vb + grp * kFV;
      nvw = min(kFV, ve - va);
      break;
    }
    grp -= ng;
  }
  if (nvw <= 0) return;
  // Runs of voxels along y when the view's depth (den) changes faster along x than
  // along y, along x otherwise: along the direction closer to the rays, consecutive
  // voxels project into the same detector cell, and the lanes of one wave (which
  // take consecutive voxels of a run) would add into that one LDS word together.
  // Across the rays they spread over the tile's columns.  rc: the coordinate a run
  // walks (0: x, 1: y); the other is the row's fixed coordinate.
  const bool ym = fabs(proj[12 * va]) > fabs(proj[12 * va + 1]);
  const int rc = ym ? 1 : 0;
  const int nzs = (g.nz + kFZS - 1) / kFZS;
  Gf += (size_t)smp * g.nx * g.ny * nzs * kFZS;
  const int ti = tile % tiles_u, tj = tile / tiles_u;
  const int i0 = ti * kFTI, i1 = min(g.nu, i0 + kFTI);
  const int j0 = tj * kFTJ, j1 = min(g.nv, j0 + kFTJ);
  if (threadIdx.x < 16 * kFV) {
    const int w = threadIdx.x >> 4, k = (threadIdx.x >> 2) & 3, c = threadIdx.x & 3;
    if (w < nvw) {
      const double* P = proj + 12 * (va + w);
      const double den = P[c], nu = P[4 + c], nvv = P[8 + c];
      double val;
      if (k == 0) val = nu - (i0 - 1) * den;        // i* >= i0 - 1
      else if (k == 1) val = i1 * den - nu;         // i* <  i1
      else if (k == 2) val = nvv - (j0 - 1) * den;  // j* >= j0 - 1
      else val = j1 * den - nvv;                    // j* <  j1
      sL[w][k][c] = val;
      if (c == rc) sNegInvA[w][k] = val != 0.0 ? -1.0 / val : 0.0;
    }
  }
  for (int q = threadIdx.x; q < kFV * kFW * kFH; q += blockDim.x) {
    (&sAB[0][0])[q] = 0ull;
    (&sCE[0][0])[q] = 0ull;
  }
  __syncthreads();
  // z-layers (16 slices each) whose box can reach the window of any of the views
  for (int zs = threadIdx.x; zs < nzs; zs += blockDim.x) {
    const double zlo = zs * kFZS, zhi = min(g.nz - 1, zs * kFZS + kFZS - 1);
    bool any = false;
    for (int w = 0; w < nvw; ++w) {
      bool on = true;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double* L = sL[w][k];
        const double mxl = fmax(0.0, L[0] * (g.nx - 1)) + fmax(0.0, L[1] * (g.ny - 1)) +
                           fmax(L[2] * zlo, L[2] * zhi) + L[3];
        if (mxl < -1e-6 * fabs(L[3]) - 1e-6) on = false;
      }
      any = any || on;
    }
    sLayerOn[zs] = any;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int n = 0;
    for (int zs = 0; zs < nzs; ++zs)
      if (sLayerOn[zs]) sLayer[n++] = zs;
    sNL = n;
  }
  __syncthreads();
  const int nfix = ym ? g.nx : g.ny, nrun = ym ? g.ny : g.nx;
  const int nrows = sNL * nfix;
  const float gabs = __uint_as_float(gmax_bits[smp]);
  // per view: the quantum S, 1/sqrt(S) (the general forms scale their
  // coordinates by it) and the scaled z-steps of den, num_u and num_v
  float S[kFV], sinv[kFV], zstep_d[kFV], zstep_u[kFV], zstep_v[kFV];
#pragma unroll
  for (int w = 0; w < kFV; ++w) {
    const float gmax = w < nvw ? gabs * rmax2[va + w] : 0.f;
    S[w] = gmax > 0.f ? qmax / gmax : 0.f;
    const double si = S[w] > 0.f ? 1.0 / sqrt((double)S[w]) : 1.0;   // S = 0: every term is zero anyway
    const double* P = proj + 12 * (va + (w < nvw ? w : 0));
    sinv[w] = (float)si;
    zstep_d[w] = (float)(P[2] * si);
    zstep_u[w] = (float)(P[6] * si);
    zstep_v[w] = (float)(P[10] * si);
  }
  for (int r0 = 0; r0 < nrows; r0 += kFROWS) {
    if (threadIdx.x == 0) sCount = 0;
    __syncthreads();
    // 1. rows of this batch (layer and fixed coordinate) whose interval along the
    // run coordinate may meet one of the frusta (written below for runs along x)
    for (int r = r0 + threadIdx.x; r < min(nrows, r0 + kFROWS); r += blockDim.x) {
      const int li = r / nfix, fc = r - li * nfix;
      const int zs = sLayer[li];
      const double zlo = zs * kFZS, zhi = min(g.nz - 1, zs * kFZS + kFZS - 1);
      double ulo = 1e30, uhi = -1e30;
      for (int w = 0; w < nvw; ++w) {
        double xlo = 0.0, xhi = nrun - 1;
        bool empty = false;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double* L = sL[w][k];
          const double a = L[rc];
          const double c0 = fma(L[1 - rc], (double)fc, L[3]);
          const double cm = fmax(fma(L[2], zlo, c0), fma(L[2], zhi, c0));
          // L_k = a x + cm >= -eta up to xb: eta = 0.01 in L's units (pixel x den)
          // keeps at least 0.01 pixel of slack (den <= 1) over the per-voxel float
          // test, whose error stays near 1e-5 pixel
          const double xb = (cm + 0.01) * sNegInvA[w][k];
          if (a > 0.0) xlo = fmax(xlo, ceil(xb));
          else if (a < 0.0) xhi = fmin(xhi, floor(xb));
          else if (cm < -0.01) empty = true;
        }
        if (!empty && xlo <= xhi) {
          ulo = fmin(ulo, xlo);
          uhi = fmax(uhi, xhi);
        }
      }
      if (ulo <= uhi) {
        const int slot = atomicAdd(&sCount, 1);
        sRow[slot] = fc;
        sLay[slot] = (unsigned char)zs;
        sXlo[slot] = (int)ulo;
        sPre[slot] = (int)(uhi - ulo) + 1;   // length for now
      }
    }
    __syncthreads();
    const int cnt = sCount;
    // 2. exclusive prefix of the run lengths (4 entries per thread)
    int loc[4], sum = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = threadIdx.x * 4 + e;
      loc[e] = idx < cnt ? sPre[idx] : 0;
      sum += loc[e];
    }
    int run = block_exclusive_scan_256(sum, sScan);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = threadIdx.x * 4 + e;
      if (idx < cnt) sPre[idx] = run;
      run += loc[e];
    }
    if (threadIdx.x == 255) sPre[cnt] = run;   // total (thread 255 holds the last entries)
    __syncthreads();
    const int total = sPre[cnt];
    // 3. flattened items: (row, x) -> a 16-voxel z-segment, projected on every view.
    // Each wave takes a contiguous quarter of the items, 64 consecutive ones per
    // pass, so a lane's next item lies 64 further on: its row is found once by
    // bisection and then advanced by a short forward scan (rows hold ~15-30 items).
    const int per_wave = (total + 3) >> 2;
    const int qa = (threadIdx.x >> 6) * per_wave, qb = min(total, qa + per_wave);
    // the items for one form F (kConeMixed takes the sample's form at run time:
    // one uniform branch per batch, the same arithmetic as the form's own kernel)
    auto items = [&](auto form_tag) __attribute__((always_inline)) {
    constexpr int F = decltype(form_tag)::value;
    int lo = -1;
    for (int q = qa + (threadIdx.x & 63); q < qb; q += 64) {
      if (lo < 0) {
        int l = 0, h = cnt - 1;
        while (l < h) {                       // last row with sPre[row] <= q
          const int mid = (l + h + 1) >> 1;
          if (sPre[mid] <= q) l = mid; else h = mid - 1;
        }
        lo = l;
      } else {
        while (sPre[lo + 1] <= q) ++lo;       // sPre[cnt] = total ends the scan
      }
      const int fc = sRow[lo], rcoord = sXlo[lo] + (q - sPre[lo]);
      const int iy = ym ? rcoord : fc, ix = ym ? fc : rcoord;
      const int zs = sLay[lo];
      const int iz0 = zs * kFZS;
      // the segment's brick: four 16-byte loads from one address (slices past the
      // last one hold zeros); column indices stay below 2^29 (the plan bounds the
      // volume), the byte offset is formed in 64 bits
      const unsigned col = (unsigned)(zs * g.ny + iy) * (unsigned)g.nx + (unsigned)ix;
      const float4* brick = reinterpret_cast<const float4*>(Gf) + (size_t)col * (kFZS / 4);
      float gv[kFZS];
#pragma unroll
      for (int k = 0; k < kFZS / 4; ++k) {
        const float4 q4 = brick[k];
        gv[4 * k] = q4.x;
        gv[4 * k + 1] = q4.y;
        gv[4 * k + 2] = q4.z;
        gv[4 * k + 3] = q4.w;
      }
      for (int w = 0; w < nvw; ++w) {
        unsigned long long* ab = sAB[w];
        unsigned long long* ce = sCE[w];
        if constexpr (F == kConeZinv) {
          const ColumnMapZ c = column_map_z(proj + 12 * (va + w), ix, iy, iz0);
          const int li = c.i - (i0 - 1);
          if ((unsigned)li > (unsigned)(i1 - i0)) continue;
          const float K = c.r2 * pick(S, w);   // (D/U)^2 S: every term stays below 2^21 (rmax2 carries a 1e-6 margin)
          const float fuc = c.fu - 0.5f;   // centred fraction, in [-1/2, 1/2]
          const unsigned jbias = kRoundMagicBits - (unsigned)(c.jv0 - (j0 - 1));
#pragma unroll
          for (int z = 0; z < kFZS; ++z) {
            const float wm = z == 0 ? c.w0m : fmaf((float)z, c.dw, c.w0m);
            const float yw = wm + kRoundMagic;
            const int lj = (int)(__float_as_uint(yw) - jbias);
            const float x = gv[z];
            if (((unsigned)lj <= (unsigned)(j1 - j0)) & (x != 0.f)) {   // one branch, not two
              const float fvc = wm - (yw - kRoundMagic);   // centred fraction of v
              const float gs = x * K;
              const float gu = gs * fuc;
              const unsigned cell = __umul24((unsigned)lj, (unsigned)kFW) + li;   // lj < 2^24: 24-bit multiply
              atomicAdd(ab + cell, pack_terms(gs + kRoundMagic, fmaf(gs, fuc, kRoundMagic)));
              atomicAdd(ce + cell, pack_terms(fmaf(gs, fvc, kRoundMagic), fmaf(gu, fvc, kRoundMagic)));
            }
          }
          continue;
        }
        const float zd = pick(zstep_d, w);
        const ColumnMapF c = column_map_fp<F == kConeQuadratic>(proj + 12 * (va + w), ix, iy, iz0, pick(sinv, w), zd,
                                                                 pick(zstep_u, w), pick(zstep_v, w));
        // kConeQuadratic: 1/den along the segment is its quadratic Taylor polynomial
        // about the segment's middle zc (remainder below (7.5 x 5e-4)^3 = 5.3e-8 of it)
        constexpr float zc = 0.5f * (kFZS - 1);
        const float dc = F == kConeQuadratic ? fmaf(zc, zd, c.den) : c.den;
        float rr0 = __builtin_amdgcn_rcpf(dc);
        rr0 = fmaf(rr0, fmaf(-dc, rr0, 1.0f), rr0);   // one Newton step: a correctly rounded start
        const float r1 = -rr0 * rr0 * zd, r2 = -r1 * rr0 * zd;   // 1/den = rr0 + r1 (z - zc) + r2 (z - zc)^2
#pragma unroll
        for (int z = 0; z < kFZS; ++z) {
          const float tz = (float)z - zc;
          const float rr = F == kConeQuadratic ? fmaf(tz, r1, fmaf(tz * tz, r2, rr0))
                           : z == 0            ? rr0
                                               : __builtin_amdgcn_rcpf(fmaf((float)z, zd, c.den));
          // nu rr = u - iu0 - 1/2 (and likewise v): one fused rounding with the
          // 1.5 * 2^23 trick gives the cell floor(u) (an exact integer u may give the
          // cell below with fraction 1: the same taps, and range checks as usual),
          // and a second fused form the centred fraction fu - 1/2 in [-1/2, 1/2]
          const float nu = z == 0 ? c.lu : fmaf((float)z, c.ldu, c.lu);
          const float nv = z == 0 ? c.lv : fmaf((float)z, c.ldv, c.lv);
          const float yu = fmaf(nu, rr, kRoundMagic), yw = fmaf(nv, rr, kRoundMagic);
          const int li = c.iu0 + (int)(__float_as_uint(yu) - kRoundMagicBits) - (i0 - 1);
          const int lj = c.jv0 + (int)(__float_as_uint(yw) - kRoundMagicBits) - (j0 - 1);
          const float x = gv[z];
          // bitwise rather than short-circuit: one branch per voxel.  Zero voxels (the
          // ReLU mask zeroes about half of a reconstruction) skip their two atomics.
          if (((unsigned)li <= (unsigned)(i1 - i0)) & ((unsigned)lj <= (unsigned)(j1 - j0)) & (x != 0.f)) {
            const float fu = fmaf(nu, rr, kRoundMagic - yu), fv = fmaf(nv, rr, kRoundMagic - yw);
            const float xr = x * rr;
            const float gs = xr * rr;
            const float gu = gs * fu;
            // Integer rounding without conversion instructions: adding 1.5 * 2^23
            // leaves round-to-nearest-even(v) in the low mantissa bits for
            // |v| < 2^22 (every term is below 2^21), and the fused forms round
            // the products gs fu, gs fv, gu fv once.
            const unsigned cell = __umul24((unsigned)lj, (unsigned)kFW) + li;   // lj < 2^24: 24-bit multiply
            atomicAdd(ab + cell, pack_terms(fmaf(xr, rr, kRoundMagic), fmaf(gs, fu, kRoundMagic)));
            atomicAdd(ce + cell, pack_terms(fmaf(gs, fv, kRoundMagic), fmaf(gu, fv, kRoundMagic)));
          }
        }
      }
    }
    };
    if constexpr (FORM == kConeMixed) {
      const int fs = forms[smp];
      if (fs == kConeZinv) items(std::integral_constant<int, kConeZinv>{});
      else if (fs == kConeQuadratic) items(std::integral_constant<int, kConeQuadratic>{});
      else items(std::integral_constant<int, kConeGeneral>{});
    } else {
      items(std::integral_constant<int, FORM>{});
    }
    __syncthreads();
  }
  // decode the tiles
  auto lo32 = [](unsigned long long w) { return (long long)(int)(unsigned)(w & 0xffffffffull); };
  auto hi32 = [](unsigned long long w, long long lo) { return ((long long)w - lo) >> 32; };
  for (int w = 0; w < nvw; ++w) {
    const double inv = pick(S, w);
    const double invS = inv > 0.0 ? 1.0 / inv : 0.0;
    const unsigned long long* AB = sAB[w];
    const unsigned long long* CE = sCE[w];
    Tout* o = GgF + (size_t)(va + w) * g.nu * g.nv;
    for (int q = threadIdx.x; q < kFTI * kFTJ; q += blockDim.x) {
      const int di = q % kFTI, dj = q / kFTI;
      const int i = i0 + di, j = j0 + dj;
      if (i >= i1 || j >= j1) continue;
      const int li = di + 1, lj = dj + 1;
      // the sums of the cell itself (c), its left (l), lower (d) and lower-left (e)
      // neighbours, with centred fractions a = fu - 1/2, b = fv - 1/2:
      // (1 - fu)(1 - fv) = (1/2 - a)(1/2 - b), fu (1 - fv) = (1/2 + a)(1/2 - b), ...
      long long A[4], B[4], C[4], E[4];
      const int cells[4] = {lj * kFW + li, lj * kFW + li - 1, (lj - 1) * kFW + li, (lj - 1) * kFW + li - 1};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const unsigned long long ab = AB[cells[c]], ce = CE[cells[c]];
        A[c] = lo32(ab);
        B[c] = hi32(ab, A[c]);
        C[c] = lo32(ce);
        E[c] = hi32(ce, C[c]);
      }
      // exact in float64: integers below 2^40 in halves and quarters
      const double val = 0.25 * (double)(A[0] + A[1] + A[2] + A[3]) +
                         0.5 * (double)(-B[0] + B[1] - B[2] + B[3]) +
                         0.5 * (double)(-C[0] - C[1] + C[2] + C[3]) + (double)(E[0] - E[1] - E[2] + E[3]);
      o[j * g.nu + i] = from_f32<Tout>((float)(val * invS));
    }
  }
}

// the form every sample in [s_lo, s_hi] takes, or kConeMixed when they differ
static int launch_form(const Plan& p, int s_lo, int s_hi) {
  for (int smp = s_lo + 1; smp <= s_hi; ++smp)
    if (p.cone_form[smp] != p.cone_form[s_lo]) return kConeMixed;
  return p.cone_form[s_lo];
}

static hipError_t launch_cone_bp_run(const Plan& p, const void* gF, dc_dtype tF, float* f, int acc, int relu, int v0,
                                     int nv, int s_lo, int s_hi, int nzb, int form, hipStream_t s);

hipError_t launch_cone_bp(const Plan& p, const void* gF, dc_dtype tF, float* f, int acc, int relu, int v0, int nv,
                          hipStream_t s) {
  int s_lo, s_hi;
  sample_span(p, v0, nv, &s_lo, &s_hi);
  const int nzb = (p.kg.nz + kZC - 1) / kZC;
  // one launch: the samples' own form, or kConeMixed when they differ
  return launch_cone_bp_run(p, gF, tF, f, acc, relu, v0, nv, s_lo, s_hi, nzb, launch_form(p, s_lo, s_hi), s);
}

static hipError_t launch_cone_bp_run(const Plan& p, const void* gF, dc_dtype tF, float* f, int acc, int relu, int v0,
                                     int nv, int s_lo, int s_hi, int nzb, int form, hipStream_t s) {
  const int BYr = p.shape.bp_by;
  dim3 grid((p.kg.nx + kBX - 1) / kBX, (p.kg.ny + BYr - 1) / BYr, nzb * (s_hi - s_lo + 1));
  return by_dtype(tF, [&](auto t) {
    using T = decltype(t);
#define DC_BP1(ST, PI, Z, BY)                                                                                    \
  hipLaunchKernelGGL((k_cone_bp<T, ST, PI, Z, BY>), grid, dim3(kBX, BY), 0, s, (const T*)gF, f, p.kg, p.d_proj,  \
                     acc, relu, v0, nv, p.d_first, s_lo, nzb, p.d_form)
#define DC_BP(ST, PI, Z)                   \
  do {                                     \
    if (BYr == 16) DC_BP1(ST, PI, Z, 16);  \
    else DC_BP1(ST, PI, Z, 32);            \
  } while (0)
#define DC_BP_FORMS(ST, PI)                                        \
  switch (form) {                                                  \
    case kConeZinv: DC_BP(ST, PI, kConeZinv); break;               \
    case kConeQuadratic: DC_BP(ST, PI, kConeQuadratic); break;     \
    case kConeMixed: DC_BP(ST, PI, kConeMixed); break;             \
    default: DC_BP(ST, PI, kConeGeneral); break;                   \
  }
#define DC_BP_PITCH(ST)                                 \
  do {                                                  \
    if (p.bp_pitch == 64) {                             \
      DC_BP_FORMS(ST, 64);                              \
    } else {                                            \
      DC_BP_FORMS(ST, 128);                             \
    }                                                   \
  } while (0)
    switch (p.bp_pitch == 64 || p.bp_pitch == 128 ? p.bp_stage : 0) {
      case 4: DC_BP_PITCH(4); break;
      case 8: DC_BP_PITCH(8); break;
      case 12: DC_BP_PITCH(12); break;
      case 16: DC_BP_PITCH(16); break;
      default: DC_BP(0, 64, kConeGeneral); break;
    }
#undef DC_BP_PITCH
#undef DC_BP_FORMS
#undef DC_BP
#undef DC_BP1
    return hipGetLastError();
  });
}

hipError_t launch_cone_fp(const Plan& p, const float* Gf, const float* f_relu, void* GgF, dc_dtype tF, int v0,
                          int nv, hipStream_t s) {
  const int TIr = p.shape.fp_ti;
  const int tiles_u = (p.kg.nu + TIr - 1) / TIr, tiles_v = (p.kg.nv + kFTJ - 1) / kFTJ;
  int s_lo, s_hi;
  sample_span(p, v0, nv, &s_lo, &s_hi);
  const int n_smp = s_hi - s_lo + 1;
  unsigned* gmax = p.d_scratch + p.n_views;   // one word per sample
  hipError_t e = launch_zero_u32(gmax + s_lo, n_smp, s);
  if (e != hipSuccess) return e;
  const size_t n = (size_t)p.kg.nx * p.kg.ny * p.kg.nz;
  const size_t ncol = (size_t)p.kg.nx * p.kg.ny * ((p.kg.nz + kFZS - 1) / kFZS);
  const int blocks = (int)std::min<size_t>(4096, (ncol + 255) / 256);
  hipLaunchKernelGGL(k_vol_brick, dim3(blocks, n_smp), dim3(256), 0, s, Gf + s_lo * n,
                     f_relu ? f_relu + s_lo * n : nullptr, p.kg.nx, p.kg.ny, p.kg.nz, gmax + s_lo,
                     p.d_masked + s_lo * ncol * kFZS);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int n_tiles = tiles_u * tiles_v;
  return by_dtype(tF, [&](auto t) {
    using T = decltype(t);
    const float* src = p.d_masked;
    // one launch: the samples' own form, or kConeMixed when they differ
    int ng = 0;
    for (int smp = s_lo; smp <= s_hi; ++smp) {
      const int vb = std::max(v0, p.first[smp]), ve = std::min(v0 + nv, p.first[smp + 1]);
      ng += (std::max(0, ve - vb) + kFV - 1) / kFV;
    }
    if (ng > 0) {
      const dim3 grid(8 * ((n_tiles + 7) / 8) * ng);
#define DC_FP1(Z, TI)                                                                                        \
  hipLaunchKernelGGL((k_cone_fp<T, Z, TI>), grid, dim3(256), 0, s, src, (T*)GgF, p.kg, p.d_proj, p.d_rmax2, v0, \
                     nv, tiles_u, n_tiles, p.cone_qmax, gmax, p.d_first, s_lo, s_hi, ng, p.d_form)
#define DC_FP(Z)                                  \
  do {                                            \
    if (TIr == 16) DC_FP1(Z, 16);                 \
    else if (TIr == 24) DC_FP1(Z, 24);            \
    else DC_FP1(Z, 20);                           \
  } while (0)
      switch (launch_form(p, s_lo, s_hi)) {
        case kConeZinv: DC_FP(kConeZinv); break;
        case kConeQuadratic: DC_FP(kConeQuadratic); break;
        case kConeMixed: DC_FP(kConeMixed); break;
        default: DC_FP(kConeGeneral); break;
      }
#undef DC_FP
#undef DC_FP1
      const hipError_t e2 = hipGetLastError();
      if (e2 != hipSuccess) return e2;
    }
    return hipSuccess;
  });
}

}  // namespace dc
