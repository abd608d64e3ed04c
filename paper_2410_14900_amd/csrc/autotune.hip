// The autotuner of the kernels' work shapes (dc_plan_autotune): every candidate
// value of each knob is timed on the plan's own geometry, on a sample of its
// views, and the fastest is kept.  The knobs are independent (each belongs to one
// stage), so the stages are tuned one after the other.  Results are cached by a
// hash of the geometry and the GPU in an optional text file, and the environment
// can fix the knobs without any timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "dc_internal.h"

namespace dc {

// seeded values in [lo, hi): an integer hash of (index, seed), independent of the launch
__global__ void k_fill_hash(float* __restrict__ p, size_t n, unsigned seed, float lo, float hi) {
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
    unsigned h = (unsigned)q * 0x9E3779B1u ^ (unsigned)(q >> 32) * 0x85EBCA77u ^ seed;
    h ^= h >> 16;
    h *= 0x7FEB352Du;
    h ^= h >> 15;
    h *= 0x846CA68Bu;
    h ^= h >> 16;
    p[q] = lo + (hi - lo) * (float)(h >> 8) * (1.0f / 16777216.0f);
  }
}

static hipError_t fill(float* p, size_t n, unsigned seed, float lo, float hi, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_hash, dim3((unsigned)std::min<size_t>(4096, (n + 255) / 256)), dim3(256), 0, s, p, n,
                     seed, lo, hi);
  return hipGetLastError();
}

// ------------------------------------------------------------ geometry key
static uint64_t fnv1a(uint64_t h, const void* data, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

template <typename T>
static uint64_t fnv1a_value(uint64_t h, const T& v) {
  return fnv1a(h, &v, sizeof v);
}

static std::string geometry_key(const Plan& p) {
  uint64_t h = 1469598103934665603ull;
  // field by field: dc_grid has padding between its int and double members
  const dc_grid& g = p.grid;
  for (int32_t v : {g.nu, g.nv, g.n_theta, g.n_s, g.nx, g.ny, g.nz}) h = fnv1a_value(h, v);
  for (double v : {g.du, g.dv, g.ds, g.vx, g.vy, g.vz, g.ox, g.oy, g.oz}) h = fnv1a_value(h, v);
  h = fnv1a(h, &p.n_views, sizeof(p.n_views));
  h = fnv1a(h, p.first.data(), p.first.size() * sizeof(int));
  h = fnv1a(h, p.views.data(), p.views.size() * sizeof(dc_view));
  hipDeviceProp_t prop{};
  if (hipGetDeviceProperties(&prop, p.device) == hipSuccess) {
    h = fnv1a(h, prop.gcnArchName, strnlen(prop.gcnArchName, sizeof(prop.gcnArchName)));
    h = fnv1a(h, &prop.multiProcessorCount, sizeof(prop.multiProcessorCount));
  }
  char buf[32];
  std::snprintf(buf, sizeof buf, "%016" PRIx64, h);
  return buf;
}

// ------------------------------------------------------- cache and override
static std::mutex g_tune_mu;

// "splat=7,itile=64,iangles=32,bprows=32,fptile=20" over `base`; false on a malformed entry
static bool parse_knobs(const char* text, dc_knobs* k, std::string* err) {
  std::stringstream ss(text);
  std::string item;
  while (std::getline(ss, item, ',')) {
    if (item.empty()) continue;
    const size_t eq = item.find('=');
    if (eq == std::string::npos) {
      *err = "DCFBP_KNOBS: '" + item + "' is not name=value";
      return false;
    }
    const std::string name = item.substr(0, eq);
    char* end = nullptr;
    const long v = std::strtol(item.c_str() + eq + 1, &end, 10);
    if (!end || *end != '\0' || v < 0 || v > 1024) {
      *err = "DCFBP_KNOBS: bad value in '" + item + "'";
      return false;
    }
    if (name == "splat") k->splat_angles = (int32_t)v;
    else if (name == "itile") k->interp_tile_u = (int32_t)v;
    else if (name == "iangles") k->interp_angles = (int32_t)v;
    else if (name == "bprows") k->bp_block_y = (int32_t)v;
    else if (name == "fptile") k->fp_tile_u = (int32_t)v;
    else {
      *err = "DCFBP_KNOBS: unknown knob '" + name + "'";
      return false;
    }
  }
  return true;
}

static bool cache_lookup(const char* path, const std::string& key, dc_knobs* k) {
  std::ifstream in(path);
  std::string line;
  bool found = false;
  while (std::getline(in, line)) {   // the last line for a key wins
    std::istringstream ls(line);
    std::string lk;
    dc_knobs c{};
    if (ls >> lk >> c.splat_angles >> c.interp_tile_u >> c.interp_angles >> c.bp_block_y >> c.fp_tile_u && lk == key) {
      *k = c;
      found = true;
    }
  }
  return found;
}

static void cache_store(const char* path, const std::string& key, const dc_knobs& k) {
  std::ofstream out(path, std::ios::app);
  if (out) out << key << ' ' << k.splat_angles << ' ' << k.interp_tile_u << ' ' << k.interp_angles << ' '
               << k.bp_block_y << ' ' << k.fp_tile_u << '\n';
}

// ------------------------------------------------------------------ timing
struct Sample {
  std::vector<std::pair<int, int>> ranges;   // (v0, nv)
  int last = 0;                              // one past the highest view touched
};

// Up to four evenly spaced ranges of 32 consecutive views: launches of that
// size fill the GPU as the full view range does (narrower launches favour
// smaller workgroups that lose at full size), and spread ranges see views of
// every direction.
static Sample sample_views(int V) {
  Sample s;
  const int L = std::min(32, V);
  const int R = std::min(4, (V + L - 1) / L);
  for (int i = 0; i < R; ++i) {
    const int v0 = R > 1 ? (int)((long long)i * (V - L) / (R - 1)) : 0;
    s.ranges.emplace_back(v0, L);
    s.last = std::max(s.last, v0 + L);
  }
  return s;
}

// fastest of three timed runs of `run` (after one warm-up), in ms
template <typename F>
static hipError_t time_it(hipStream_t s, F&& run, double* ms) {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = run();
  double best = 1e300;
  for (int r = 0; r < 3 && e == hipSuccess; ++r) {
    if ((e = hipEventRecord(a, s)) != hipSuccess) break;
    if ((e = run()) != hipSuccess) break;
    if ((e = hipEventRecord(b, s)) != hipSuccess) break;
    if ((e = hipEventSynchronize(b)) != hipSuccess) break;
    float t = 0.f;
    if ((e = hipEventElapsedTime(&t, a, b)) != hipSuccess) break;
    best = std::min(best, (double)t);
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  *ms = best;
  return e;
}

struct Buffers {
  float *img = nullptr, *img2 = nullptr, *sino = nullptr, *vol = nullptr, *mask = nullptr, *vol2 = nullptr;
  ~Buffers() {
    for (float* q : {img, img2, sino, vol, mask, vol2})
      if (q) (void)hipFree(q);
  }
};

// One stage's candidate shapes: the incumbent (the plan's shape so far) is timed
// first, then each candidate is applied to the plan and timed; a candidate
// replaces the best so far only if it is faster by more than 2% (timing noise
// between launches is about 1%), and the best is returned in *best (with its
// time).  Shapes the geometry rejects (LDS) are skipped.
template <typename Run>
static hipError_t tune_stage(Plan* p, hipStream_t s, const KernelShape& incumbent,
                             const std::vector<KernelShape>& cands, Run&& run, KernelShape* best, double* best_ms) {
  *best_ms = 1e300;
  std::vector<KernelShape> order{incumbent};
  order.insert(order.end(), cands.begin(), cands.end());
  for (const KernelShape& ks : order) {
    if (set_shape(p, ks) != DC_OK) continue;
    double ms = 0.0;
    const hipError_t e = time_it(s, run, &ms);
    if (e != hipSuccess) return e;
    if (ms < (*best_ms < 1e300 ? 0.98 * *best_ms : *best_ms)) {
      *best_ms = ms;
      *best = ks;
    }
  }
  return hipSuccess;
}

dc_status autotune(Plan* p, hipStream_t s, dc_knobs* chosen, double* ms_out, int32_t* source) {
  const KernelShape start = p->shape;
  double ms[4] = {0, 0, 0, 0};
  auto finish = [&](int32_t src) {
    if (chosen) *chosen = knobs_of(p->shape);
    if (ms_out)
      for (int i = 0; i < 4; ++i) ms_out[i] = ms[i];
    if (source) *source = src;
    return DC_OK;
  };
  // 1. the environment fixes the knobs
  if (const char* env = std::getenv("DCFBP_KNOBS")) {
    dc_knobs k = knobs_of(p->shape);
    std::string err;
    if (!parse_knobs(env, &k, &err)) {
      set_error(err);
      return DC_EINVAL;
    }
    const dc_status st = set_shape(p, shape_of(k));
    if (st != DC_OK) return st;
    return finish(2);
  }
  // 2. an earlier result for this geometry and GPU
  const char* cache = std::getenv("DCFBP_TUNE_CACHE");
  const std::string key = geometry_key(*p);
  if (cache && *cache) {
    dc_knobs k{};
    bool hit;
    {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      hit = cache_lookup(cache, key, &k);
    }
    if (hit && set_shape(p, shape_of(k)) == DC_OK) return finish(1);
  }
  // 3. time the candidates
  const Sample smp = sample_views(p->n_views);
  const KGrid& g = p->kg;
  const size_t npix = (size_t)g.nu * g.nv, nbin = (size_t)g.n_theta * g.n_s;
  const size_t nvol = (size_t)p->n_samples * g.nx * g.ny * g.nz;
  Buffers b;
  hipError_t e = hipSuccess;
  auto need = [&](float** q, size_t n) {
    if (e == hipSuccess) e = hipMalloc((void**)q, n * sizeof(float));
  };
  need(&b.img, smp.last * npix);
  need(&b.img2, smp.last * npix);
  need(&b.sino, smp.last * nbin);
  need(&b.vol, nvol);
  need(&b.mask, nvol);
  need(&b.vol2, nvol);
  if (e == hipSuccess) e = fill(b.img, smp.last * npix, 1u, 0.f, 1.f, s);
  if (e == hipSuccess) e = fill(b.sino, smp.last * nbin, 2u, -1.f, 1.f, s);
  if (e == hipSuccess) e = fill(b.vol, nvol, 3u, -1.f, 1.f, s);
  if (e == hipSuccess) e = fill(b.mask, nvol, 4u, -0.5f, 1.f, s);   // about two thirds kept by the ReLU mask
  if (e != hipSuccess) {
    set_error(std::string("autotune buffers: ") + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? DC_ENOMEM : DC_EHIP;
  }
  const float scale_r = (float)(p->grid.du * p->grid.dv / p->grid.ds), scale_b = (float)(M_PI / p->grid.n_theta);
  auto over_ranges = [&](auto&& stage) {
    return [&, stage]() -> hipError_t {
      for (const auto& r : smp.ranges) {
        const hipError_t x = stage(r.first, r.second);
        if (x != hipSuccess) return x;
      }
      return hipSuccess;
    };
  };
  KernelShape cur = start, best;
  double best_ms = 0.0;
  // splat angles per workgroup
  {
    std::vector<KernelShape> c;
    for (int kc = 2; kc <= 8; ++kc) {
      KernelShape k = cur;
      k.splat_kc = kc;
      c.push_back(k);
    }
    e = tune_stage(p, s, cur, c, over_ranges([&](int v0, int nv) {
                     return launch_splat(*p, b.img, DC_F32, true, scale_r, b.sino, DC_F32, v0, nv, s);
                   }),
                   &best, &best_ms);
    if (e == hipSuccess && best_ms < 1e300) {
      cur.splat_kc = best.splat_kc;
      ms[0] = best_ms;
    }
  }
  // detector-BP tile width x angles per chunk
  if (e == hipSuccess) {
    std::vector<KernelShape> c;
    for (int tx : {32, 64})
      for (int kc : {16, 32, 64}) {
        KernelShape k = cur;
        k.interp_tx = tx;
        k.interp_kc = kc;
        c.push_back(k);
      }
    e = tune_stage(p, s, cur, c, over_ranges([&](int v0, int nv) {
                     return launch_interp(*p, b.sino, DC_F32, false, scale_b, b.img2, DC_F32, v0, nv, s);
                   }),
                   &best, &best_ms);
    if (e == hipSuccess && best_ms < 1e300) {
      cur.interp_tx = best.interp_tx;
      cur.interp_kc = best.interp_kc;
      ms[1] = best_ms;
    }
  }
  // cone-BP block rows
  if (e == hipSuccess) {
    std::vector<KernelShape> c;
    for (int by : {16, 32}) {
      KernelShape k = cur;
      k.bp_by = by;
      c.push_back(k);
    }
    e = tune_stage(p, s, cur, c, over_ranges([&](int v0, int nv) {
                     return launch_cone_bp(*p, b.img, DC_F32, b.vol2, 0, 1, v0, nv, s);
                   }),
                   &best, &best_ms);
    if (e == hipSuccess && best_ms < 1e300) {
      cur.bp_by = best.bp_by;
      ms[2] = best_ms;
    }
  }
  // cone-FP tile width
  if (e == hipSuccess) {
    std::vector<KernelShape> c;
    for (int ti : {16, 20, 24}) {
      KernelShape k = cur;
      k.fp_ti = ti;
      c.push_back(k);
    }
    e = tune_stage(p, s, cur, c, over_ranges([&](int v0, int nv) {
                     return launch_cone_fp(*p, b.vol, b.mask, b.img2, DC_F32, v0, nv, s);
                   }),
                   &best, &best_ms);
    if (e == hipSuccess && best_ms < 1e300) {
      cur.fp_ti = best.fp_ti;
      ms[3] = best_ms;
    }
  }
  if (e != hipSuccess) {
    (void)set_shape(p, start);
    set_error(std::string("autotune: ") + hipGetErrorString(e));
    return DC_EHIP;
  }
  const dc_status st = set_shape(p, cur);
  if (st != DC_OK) {
    (void)set_shape(p, start);
    return st;
  }
  if (cache && *cache) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    cache_store(cache, key, knobs_of(p->shape));
  }
  return finish(0);
}

}  // namespace dc
