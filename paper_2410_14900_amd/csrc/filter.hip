// Shift-variant filtering in the sinogram domain (paper eqs. 7, 10, 11):
//
//   Q = D R,   P = W Q,   H = D P,     W = M c_geo  (ANALYTIC)  or  W = M  (RAW)
//   c_geo(k, m) = -| t.n_mu / (4 pi^2 D) + s_m t.l_z / (4 pi^2 D^2) |
//
// D is the zero-padded central difference along s.  The adjoint gives
// GP = D^T GH = -D GH, GM = GP Q c_geo and GR = D^T (W GP).
//
// The stage is bound by its 12 bytes/bin of HBM traffic, so the kernels are
// built around the loads: one workgroup takes kRows consecutive sinogram rows
// (rows of all views are contiguous, [V][n_theta][n_s]), a flat run of
// kRows n_s elements that starts on a multiple of kRows rows and is therefore
// aligned to 4 elements.  Every thread issues all of its 4-element vector loads
// of both inputs (R and M; GH, R and the optional M and GM) before the first
// barrier, so the streams overlap; the differences then run in LDS, and the
// outputs leave as 4-element vector stores.  Rows outside the call's view range
// (at its ends, where a run straddles it) are read but never written.
#include <type_traits>

#include "dc_internal.h"

namespace dc {

static constexpr int kRows = 4;          // sinogram rows per workgroup
static constexpr int kFThreads = 256;
// NV: 4-element vectors per thread, the smallest instantiated count with
// kFThreads NV >= n_s (kRows n_s / 4 vectors per run); n_s <= 4096 gives NV <= 16

__device__ __forceinline__ float cgeo_row(const float4 vf, const float2 cs) {
  return vf.y * cs.x + vf.z * cs.y;   // t.n_mu / (4 pi^2 D)
}

// 4 consecutive storage elements at p (aligned to 4 elements) as float32
__device__ __forceinline__ float4 load4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ float4 load4(const bf16_t* p) {
  const uint2 u = *reinterpret_cast<const uint2*>(p);
  return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u), __uint_as_float(u.y << 16),
                     __uint_as_float(u.y & 0xffff0000u));
}
__device__ __forceinline__ float4 load4(const _Float16* p) {
  const uint2 u = *reinterpret_cast<const uint2*>(p);
  const _Float16* h = reinterpret_cast<const _Float16*>(&u);
  return make_float4((float)h[0], (float)h[1], (float)h[2], (float)h[3]);
}
__device__ __forceinline__ void store4(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }
template <typename T>
__device__ __forceinline__ void store4(T* p, float4 v) {   // 16-bit storage: one 8-byte store
  T h[4] = {from_f32<T>(v.x), from_f32<T>(v.y), from_f32<T>(v.z), from_f32<T>(v.w)};
  *reinterpret_cast<uint2*>(p) = *reinterpret_cast<const uint2*>(h);
}

__device__ __forceinline__ float comp(const float4& v, int c) {
  return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w;
}

// The run of one workgroup: flat elements [base, base + kRows n_s) of the stack,
// rows [row0, row0 + kRows).  Vector q covers elements base + 4q .. base + 4q + 3.
struct Run {
  size_t base;
  int row0;
  int n;            // kRows n_s
};

__device__ __forceinline__ Run run_of(const KGrid& g, int v0) {
  const int first = (v0 * g.n_theta) / kRows * kRows;
  Run r;
  r.row0 = first + blockIdx.x * kRows;
  r.base = (size_t)r.row0 * g.n_s;
  r.n = kRows * g.n_s;
  return r;
}

// element e of a run: its row within the run and its bin
__device__ __forceinline__ void split(int e, int ns, float inv_ns, int* row, int* m) {
  // (e + 1/2) / ns lies at least 1/(2 ns) from an integer; the float product's
  // error is below 1e-6 for e < 4 n_s
  *row = (int)(((float)e + 0.5f) * inv_ns);
  *m = e - *row * ns;
}

// Per-row filter constants of a run in LDS (read by element rows, a runtime index):
// valid: row row0 + r lies in the call's rows [lo, hi); a = t.n_mu / (4 pi^2 D),
// w = t.l_z / (4 pi^2 D^2) of the row's view and angle.  Written by threads < kRows.
struct RowConst {
  float a[kRows], w[kRows];
  int valid[kRows];
};

__device__ __forceinline__ void row_consts(const KGrid& g, const Run& run, int lo, int hi,
                                           const float4* __restrict__ viewf, const float2* __restrict__ trig,
                                           RowConst* rc) {
  if (threadIdx.x < kRows) {
    const int r = threadIdx.x, row = run.row0 + r;
    rc->valid[r] = row >= lo && row < hi;
    const int rr = min(max(row, lo), hi - 1);   // rows outside the range take a valid row's constants
    const int v = rr / g.n_theta, k = rr - v * g.n_theta;
    const float4 vf = viewf[v];
    rc->a[r] = cgeo_row(vf, trig[k]);
    rc->w[r] = vf.w;
  }
}

template <typename TR, typename TH, int NV>
__global__ __launch_bounds__(kFThreads) void k_filter(const TR* __restrict__ R, const float* __restrict__ M,
                                                      TH* __restrict__ H, KGrid g, const float4* __restrict__ viewf,
                                                      const float2* __restrict__ trig, int raw, int v0, int nv,
                                                      size_t total) {
  extern __shared__ float sh[];
  const Run run = run_of(g, v0);
  float* r = sh;              // [kRows n_s]
  float* pw = sh + run.n;     // [kRows n_s]
  const int ns = g.n_s, nvec = run.n / 4;
  const int lo = v0 * g.n_theta, hi = (v0 + nv) * g.n_theta;
  // 1. every load of the run first: R into registers then LDS, M into registers
  float4 rv[NV], mv[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const int q = threadIdx.x + kFThreads * j;
    if (q < nvec) {
      const size_t e = run.base + 4 * (size_t)q;
      if (e + 4 <= total) {
        rv[j] = load4(R + e);
        mv[j] = load4(M + e);
      } else {   // the stack's last run: elements past its end read as 0
        float t[4], u[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          t[c] = e + c < total ? to_f32(R[e + c]) : 0.f;
          u[c] = e + c < total ? M[e + c] : 0.f;
        }
        rv[j] = make_float4(t[0], t[1], t[2], t[3]);
        mv[j] = make_float4(u[0], u[1], u[2], u[3]);
      }
    }
  }
  __shared__ RowConst rc;
  row_consts(g, run, lo, hi, viewf, trig, &rc);
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const int q = threadIdx.x + kFThreads * j;
    if (q < nvec) *reinterpret_cast<float4*>(r + 4 * q) = rv[j];
  }
  __syncthreads();
  const float inv_ns = 1.0f / (float)ns;
  const float inv2ds = 0.5f / g.ds;
  const float s0 = -0.5f * (ns - 1) * g.ds;
  // 2. P = W (D R)
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const int q = threadIdx.x + kFThreads * j;
    if (q < nvec) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int e = 4 * q + c;
        int row, m;
        split(e, ns, inv_ns, &row, &m);
        const float rp = (m + 1 < ns) ? r[e + 1] : 0.f;
        const float rm = (m > 0) ? r[e - 1] : 0.f;
        float w = comp(mv[j], c);
        if (!raw) w *= -fabsf(fmaf(fmaf((float)m, g.ds, s0), rc.w[row], rc.a[row]));
        pw[e] = w * (rp - rm) * inv2ds;
      }
    }
  }
  __syncthreads();
  // 3. H = D P, written for the rows of the call
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const int q = threadIdx.x + kFThreads * j;
    if (q < nvec) {
      float hv[4];
      bool all = true;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int e = 4 * q + c;
        int row, m;
        split(e, ns, inv_ns, &row, &m);
        const float pp = (m + 1 < ns) ? pw[e + 1] : 0.f;
        const float pm = (m > 0) ? pw[e - 1] : 0.f;
        hv[c] = (pp - pm) * inv2ds;
        all = all && rc.valid[row];
      }
      const size_t e = run.base + 4 * (size_t)q;
      if (all && e + 4 <= total) {
        store4(H + e, make_float4(hv[0], hv[1], hv[2], hv[3]));
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          int row, m;
          split(4 * q + c, ns, inv_ns, &row, &m);
          if (rc.valid[row] && e + c < total) H[e + c] = from_f32<TH>(hv[c]);
        }
      }
    }
  }
}

template <typename TH, typename TR, int NV>
__global__ __launch_bounds__(kFThreads) void k_filter_adj(const TH* __restrict__ GH, const TR* __restrict__ R,
                                                          const float* __restrict__ M, float* __restrict__ GM,
                                                          int acc, float* __restrict__ GR, KGrid g,
                                                          const float4* __restrict__ viewf,
                                                          const float2* __restrict__ trig, int raw, int v0, int nv,
                                                          size_t total) {
  extern __shared__ float sh[];
  const Run run = run_of(g, v0);
  float* gh = sh;               // [kRows n_s]
  float* r = sh + run.n;        // [kRows n_s]
  float* gq = sh + 2 * run.n;   // [kRows n_s] (GR only)
  const int ns = g.n_s, nvec = run.n / 4;
  const int lo = v0 * g.n_theta, hi = (v0 + nv) * g.n_theta;
  const bool want_m = GR != nullptr, want_gm = GM != nullptr && acc;
  // 1. every load first: GH and R to LDS, M (for GR) and GM (when accumulating) in registers
  float4 mv[NV], gmv[NV];
  {
    float4 ghv[NV], rv[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int q = threadIdx.x + kFThreads * j;
      if (q < nvec) {
        const size_t e = run.base + 4 * (size_t)q;
        if (e + 4 <= total) {
          ghv[j] = load4(GH + e);
          rv[j] = load4(R + e);
          if (want_m) mv[j] = load4(M + e);
          if (want_gm) gmv[j] = load4(GM + e);
        } else {
          float t[4], u[4], w[4], x[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const bool in = e + c < total;
            t[c] = in ? to_f32(GH[e + c]) : 0.f;
            u[c] = in ? to_f32(R[e + c]) : 0.f;
            w[c] = in && want_m ? M[e + c] : 0.f;
            x[c] = in && want_gm ? GM[e + c] : 0.f;
          }
          ghv[j] = make_float4(t[0], t[1], t[2], t[3]);
          rv[j] = make_float4(u[0], u[1], u[2], u[3]);
          mv[j] = make_float4(w[0], w[1], w[2], w[3]);
          gmv[j] = make_float4(x[0], x[1], x[2], x[3]);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int q = threadIdx.x + kFThreads * j;
      if (q < nvec) {
        *reinterpret_cast<float4*>(gh + 4 * q) = ghv[j];
        *reinterpret_cast<float4*>(r + 4 * q) = rv[j];
      }
    }
  }
  __shared__ RowConst rc;
  row_consts(g, run, lo, hi, viewf, trig, &rc);
  __syncthreads();
  const float inv_ns = 1.0f / (float)ns;
  const float inv2ds = 0.5f / g.ds;
  const float s0 = -0.5f * (ns - 1) * g.ds;
  // 2. GP = -D GH, GM (+)= GP Q c_geo, and W GP for GR
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const int q = threadIdx.x + kFThreads * j;
    if (q < nvec) {
      float gmo[4];
      bool all = true;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int e = 4 * q + c;
        int row, m;
        split(e, ns, inv_ns, &row, &m);
        const float gp = (((m > 0) ? gh[e - 1] : 0.f) - ((m + 1 < ns) ? gh[e + 1] : 0.f)) * inv2ds;
        const float qq = (((m + 1 < ns) ? r[e + 1] : 0.f) - ((m > 0) ? r[e - 1] : 0.f)) * inv2ds;
        const float cg = raw ? 1.f : -fabsf(fmaf(fmaf((float)m, g.ds, s0), rc.w[row], rc.a[row]));
        const float gm = gp * qq * cg;
        gmo[c] = want_gm ? comp(gmv[j], c) + gm : gm;
        if (want_m) gq[e] = comp(mv[j], c) * cg * gp;
        all = all && rc.valid[row];
      }
      if (GM) {
        const size_t e = run.base + 4 * (size_t)q;
        if (all && e + 4 <= total) {
          store4(GM + e, make_float4(gmo[0], gmo[1], gmo[2], gmo[3]));
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            int row, m;
            split(4 * q + c, ns, inv_ns, &row, &m);
            if (rc.valid[row] && e + c < total) GM[e + c] = gmo[c];
          }
        }
      }
    }
  }
  if (!want_m) return;
  __syncthreads();
  // 3. GR = D^T (W GP)
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const int q = threadIdx.x + kFThreads * j;
    if (q < nvec) {
      float o[4];
      bool all = true;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int e = 4 * q + c;
        int row, m;
        split(e, ns, inv_ns, &row, &m);
        o[c] = (((m > 0) ? gq[e - 1] : 0.f) - ((m + 1 < ns) ? gq[e + 1] : 0.f)) * inv2ds;
        all = all && rc.valid[row];
      }
      const size_t e = run.base + 4 * (size_t)q;
      if (all && e + 4 <= total) {
        store4(GR + e, make_float4(o[0], o[1], o[2], o[3]));
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          int row, m;
          split(4 * q + c, ns, inv_ns, &row, &m);
          if (rc.valid[row] && e + c < total) GR[e + c] = o[c];
        }
      }
    }
  }
}

// workgroups covering the call's rows [v0 n_theta, (v0 + nv) n_theta) in runs of
// kRows rows starting on a multiple of kRows
static int filter_blocks(const Plan& p, int v0, int nv) {
  const int first = (v0 * p.kg.n_theta) / kRows * kRows;
  const int end = (v0 + nv) * p.kg.n_theta;
  return (end - first + kRows - 1) / kRows;
}

// calls f with std::integral_constant<int, NV> for the smallest NV in {1, 2, 3, 4, 6, 8, 12, 16}
// holding n_s vectors per kFThreads threads
template <typename F>
static hipError_t by_vectors(int n_s, F&& f) {
  const int need = (n_s + kFThreads - 1) / kFThreads;
  if (need <= 1) return f(std::integral_constant<int, 1>{});
  if (need <= 2) return f(std::integral_constant<int, 2>{});
  if (need <= 3) return f(std::integral_constant<int, 3>{});
  if (need <= 4) return f(std::integral_constant<int, 4>{});
  if (need <= 6) return f(std::integral_constant<int, 6>{});
  if (need <= 8) return f(std::integral_constant<int, 8>{});
  if (need <= 12) return f(std::integral_constant<int, 12>{});
  return f(std::integral_constant<int, 16>{});
}

hipError_t launch_filter(const Plan& p, const void* R, dc_dtype tR, const float* M, int raw, void* H,
                         dc_dtype tH, int v0, int nv, hipStream_t s) {
  dim3 grid(filter_blocks(p, v0, nv));
  const size_t lds = 2 * (size_t)kRows * p.kg.n_s * sizeof(float);
  const size_t total = (size_t)p.n_views * p.kg.n_theta * p.kg.n_s;
  return by_dtype(tR, [&](auto tr) {
    using TR = decltype(tr);
    return by_dtype(tH, [&](auto th) {
      using TH = decltype(th);
      return by_vectors(p.kg.n_s, [&](auto nvc) {
        constexpr int NV = decltype(nvc)::value;
        hipLaunchKernelGGL((k_filter<TR, TH, NV>), grid, dim3(kFThreads), lds, s, (const TR*)R, M, (TH*)H, p.kg,
                           (const float4*)p.d_view, (const float2*)p.d_trig, raw, v0, nv, total);
        return hipGetLastError();
      });
    });
  });
}

hipError_t launch_filter_adjoint(const Plan& p, const void* GH, dc_dtype tH, const void* R, dc_dtype tR,
                                 const float* M, int raw, float* GM, int acc, float* GR, int v0, int nv,
                                 hipStream_t s) {
  dim3 grid(filter_blocks(p, v0, nv));
  const size_t lds = (GR ? 3 : 2) * (size_t)kRows * p.kg.n_s * sizeof(float);
  const size_t total = (size_t)p.n_views * p.kg.n_theta * p.kg.n_s;
  return by_dtype(tH, [&](auto th) {
    using TH = decltype(th);
    return by_dtype(tR, [&](auto tr) {
      using TR = decltype(tr);
      return by_vectors(p.kg.n_s, [&](auto nvc) {
        constexpr int NV = decltype(nvc)::value;
        hipLaunchKernelGGL((k_filter_adj<TH, TR, NV>), grid, dim3(kFThreads), lds, s, (const TH*)GH, (const TR*)R, M,
                           GM, acc, GR, p.kg, (const float4*)p.d_view, (const float2*)p.d_trig, raw, v0, nv, total);
        return hipGetLastError();
      });
    });
  });
}

}  // namespace dc
