// Continuous-batching render server: one device step advances every live ray
// of every admitted request by one surface interaction.
//
// All requests share one ray queue.  A ray carries, in its flag word, the
// scene it belongs to, the environment that lights it (the scene's own for a
// render, another one for a relight), its request slot, its own generation and
// its request's depth cap, so rays of requests admitted at different times,
// with different depths, scenes and environments, are traced by the same
// kernels.  Children are written with the tracer's stable compaction, so the
// rays of one request stay contiguous runs and a wave mostly walks one BVH.
// Newly admitted requests' camera rays are appended to the queue at the start
// of a step and traced in that same step.  After the step a per-slot
// histogram of the next queue tells the host which requests have no rays left.
#include <string.h>

#include "dt_queue.h"

namespace {

constexpr int TBS = 64;
constexpr int EBS = 256;

// ray flag word
constexpr uint32_t SF_INSIDE = 1u;
__device__ __host__ __forceinline__ uint32_t sf_depth(uint32_t f) { return (f >> 1) & 31u; }
__device__ __host__ __forceinline__ uint32_t sf_maxd(uint32_t f) { return (f >> 6) & 31u; }
__device__ __host__ __forceinline__ uint32_t sf_scene(uint32_t f) { return (f >> 11) & 7u; }
__device__ __host__ __forceinline__ uint32_t sf_env(uint32_t f) { return (f >> 14) & 7u; }
__device__ __host__ __forceinline__ uint32_t sf_slot(uint32_t f) { return (f >> 17) & 255u; }
__device__ __host__ __forceinline__ uint32_t sf_make(uint32_t inside, uint32_t depth, uint32_t maxd,
                                                     uint32_t scene, uint32_t env, uint32_t slot) {
  return inside | (depth << 1) | (maxd << 6) | (scene << 11) | (env << 14) | (slot << 17);
}

struct ServeTables {
  SceneDev sc[DT_SERVE_MAX_SCENES];
  EnvDev env[DT_SERVE_MAX_ENVS];
};
// the tables travel to the device as a kernel argument (k_set_tables), so a
// step queues no copy from host memory and never waits for one
static_assert(sizeof(ServeTables) <= 3584, "serving tables must fit a kernel argument");

// Per-pixel outputs of a step (pool-sized; flags / sig may be NULL) and the
// per-slot count of rays lost to a full queue.
struct ServeOut {
  float* pixels;
  int32_t* flags;
  unsigned long long* sig;
  uint32_t* slot_dropped;
};

__device__ __forceinline__ void serve_flag(const ServeOut& out, int pix, int32_t f) {
  if (out.flags && f) atomicOr(out.flags + pix, f);
}

// a ray of slot `slot` (pixel pix) was not written: the queue is full
__device__ __forceinline__ void serve_drop(const ServeOut& out, uint32_t* dropped, uint32_t slot,
                                           int pix) {
  atomicAdd(dropped, 1u);
  atomicAdd(out.slot_dropped + slot, 1u);
  serve_flag(out, pix, DT_FLAG_OVERFLOW);
}

struct ServeState {
  Counters ctr;            // count[0] = live rays of the current queue
  long long traced;        // rays intersected since the last reset
  long long dropped;
  WorkPart wp[DT_WORK_PARTS];  // traversal work cursors of the current queue
};

constexpr int SERVE_TRACE_BLOCKS = 256 * 4 * 7;

struct ServeLayout {
  size_t state, tables, part0, part1, q[2][3], hit, code, ovf, miss, total;
  int64_t cap, maxchunks;
};

ServeLayout serve_layout(int64_t cap) {
  ServeLayout L;
  L.cap = cap;
  L.maxchunks = (cap + DT_CHUNK - 1) / DT_CHUNK;
  size_t o = 0;
  L.state = o;
  o = dt_align(o + sizeof(ServeState));
  L.tables = o;
  o = dt_align(o + sizeof(ServeTables));
  L.part0 = o;
  o = dt_align(o + 8 * ((size_t)L.maxchunks + 1));
  L.part1 = o;
  o = dt_align(o + 8 * ((size_t)L.maxchunks + 1));
  for (int b = 0; b < 2; ++b)
    for (int k = 0; k < 3; ++k) {
      L.q[b][k] = o;
      o = dt_align(o + 16 * (size_t)cap);
    }
  L.hit = o;
  o = dt_align(o + 16 * (size_t)cap);
  L.code = o;
  o = dt_align(o + 4 * (size_t)cap);
  L.ovf = o;
  o = dt_align(o + 8 * (size_t)SERVE_TRACE_BLOCKS * TBS * (DT_STACK - DT_STACK_LDS));
  L.miss = o;  // misses lit by one MLP environment (rebuilt per environment)
  o = dt_align(o + 4 * (size_t)cap);
  L.total = o;
  return L;
}

Gen serve_gen(char* W, const ServeLayout& L, int b) {
  Gen g;
  g.o = (float4*)(W + L.q[b][0]);
  g.d = (float4*)(W + L.q[b][1]);
  g.w = (float4*)(W + L.q[b][2]);
  g.hit = (float4*)(W + L.hit);
  g.code = (uint32_t*)(W + L.code);
  g.child = nullptr;
  return g;
}

__global__ void k_set_tables(ServeTables T, ServeTables* Td) {
  // word-by-word copy of the argument into the workspace
  const uint32_t* src = (const uint32_t*)&T;
  uint32_t* dst = (uint32_t*)Td;
  for (int k = threadIdx.x; k < (int)(sizeof(ServeTables) / 4); k += blockDim.x) dst[k] = src[k];
}

__global__ void k_serve_reset(ServeState* st, unsigned long long* p0, unsigned long long* p1,
                              int64_t np) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i == 0) {
    Counters& c = st->ctr;
    for (int g = 0; g < DT_MAX_DEPTH + 2; ++g) c.count[g] = c.nrefl[g] = c.hits[g] = c.nmiss[g] = 0;
    for (int x = 0; x < DT_WORK_PARTS; ++x) st->wp[x].next = 0;
    c.dropped = 0;
    st->traced = 0;
    st->dropped = 0;
  }
  for (; i < np; i += (int64_t)gridDim.x * blockDim.x) {
    p0[i] = 0ull;
    p1[i] = 0ull;
  }
}

// camera rays of one admitted request, appended after the live rays
__global__ void k_serve_raygen(Gen q, ServeState* st, int64_t prefix, CamDev c, uint32_t flags,
                               int64_t cap, ServeOut out) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t n = (int64_t)c.W * c.H;
  if (r >= n) return;
  int64_t i = (int64_t)st->ctr.count[0] + prefix + r;
  int x, y;
  v3 d = camera_ray(c, r, x, y);
  int pix = (int)(c.pixel_offset + (int64_t)y * c.W + x);
  if (i >= cap) {
    serve_drop(out, &st->ctr.dropped, sf_slot(flags), pix);
    return;
  }
  q.o[i] = make_float4(c.eye[0], c.eye[1], c.eye[2], __int_as_float(-1));
  q.d[i] = make_float4(d.x, d.y, d.z, __int_as_float(pix));
  q.w[i] = make_float4(1.f, 1.f, 1.f, __int_as_float((int)flags));
}

// an admitted request's image, flags and signatures start at zero, and so
// does its slot's drop count
__global__ void k_serve_clear(ServeOut out, int64_t off, int64_t np, uint32_t slot) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < np;
       i += (int64_t)gridDim.x * blockDim.x) {
    out.pixels[3 * (off + i)] = 0.f;
    out.pixels[3 * (off + i) + 1] = 0.f;
    out.pixels[3 * (off + i) + 2] = 0.f;
    if (out.flags) out.flags[off + i] = 0;
    if (out.sig) out.sig[off + i] = 0ull;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out.slot_dropped[slot] = 0u;
}

__global__ void k_serve_admit_count(ServeState* st, int64_t added, int64_t cap) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int64_t n = (int64_t)st->ctr.count[0] + added;
    st->ctr.count[0] = (uint32_t)(n < cap ? n : cap);
  }
}

__global__ void __launch_bounds__(TBS, 7) k_serve_trace(const ServeTables* T, Gen q, ServeState* st,
                                                     unsigned long long* part, ServeOut out,
                                                     uint2* ovf) {
  __shared__ uint2 stk[DT_STACK_LDS * TBS];
  __shared__ LeafQueue lq;
  uint2* gstk = ovf + (size_t)(blockIdx.x * TBS + threadIdx.x) * (DT_STACK - DT_STACK_LDS);
  Counters* ctr = &st->ctr;
  const uint32_t n = ctr->count[0];
  const int lane = threadIdx.x & 63;
  const uint32_t nb = (n + 63u) / 64u;
  const uint32_t x0 = blockIdx.x % (unsigned)DT_WORK_PARTS;
  uint32_t p = x0, batch = 0;
  while (claim_batch(st->wp, nb, x0, p, batch)) {
    const uint32_t base = batch * 64u;
    uint32_t i = base + lane;
    const bool active = i < n;
    bool has_r = false, has_t = false;
    float4 o4 = make_float4(0.f, 0.f, 0.f, __int_as_float(-1)), d4 = make_float4(0.f, 0.f, 1.f, 0.f);
    if (active) {
      o4 = q.o[i];
      d4 = q.d[i];
    }
    // lanes without a ray take scene 0's tree (they only ride along)
    uint32_t fl = active ? (uint32_t)__float_as_int(q.w[i].w) : 0u;
    const SceneDev& sc = T->sc[sf_scene(fl)];
    bool ovf = false;
    const Hit h = closest_hit_wave<DT_STACK_LDS, true, true>(sc.bvh, active, xyz(o4), xyz(d4),
                                                             __float_as_int(o4.w), sc.t_eps,
                                                             stk + threadIdx.x, TBS, gstk,
                                                             DT_STACK - DT_STACK_LDS, lq, &ovf);
    if (active) {
      // reloaded rather than kept in registers through the traversal
      o4 = q.o[i];
      d4 = q.d[i];
      const float4 w4 = q.w[i];
      fl = (uint32_t)__float_as_int(w4.w);
      v3 o = xyz(o4), d = xyz(d4), W = xyz(w4);
      int pix = __float_as_int(d4.w);
      q.hit[i] = make_float4(h.t, __int_as_float(h.tri), h.b1, h.b2);
      uint32_t code = 0;
      int32_t pf = ovf ? DT_FLAG_STACK : 0;
      if (h.tri < 0) {
        if (fl & SF_INSIDE) pf |= DT_FLAG_LEAK;
        // equirect lookups here; MLP-lit misses are listed per environment
        // after the trace and evaluated on the matrix cores
        const EnvDev& env = T->env[sf_env(fl)];
        if (env.kind == DT_ENV_EQUIRECT) {
          v3 E = env_equirect(env, d);
          atomicAdd(out.pixels + 3 * pix, W.x * E.x);
          atomicAdd(out.pixels + 3 * pix + 1, W.y * E.y);
          atomicAdd(out.pixels + 3 * pix + 2, W.z * E.z);
        }
      } else {
        HitGeo geo = load_geo(sc, h.tri);
        Shade s = shade(sc, geo, o, d, h.t, h.b1, h.b2, 0u);
        code = s.code;
        if (code & C_DEGEN) pf |= DT_FLAG_DEGEN;
        if (code & C_GRAZE) pf |= DT_FLAG_GRAZING;
        if (code & C_TIRB) pf |= DT_FLAG_TIRB;
        if (sf_depth(fl) >= sf_maxd(fl)) {
          code |= C_TRUNC;
          pf |= DT_FLAG_TRUNC;
        } else {
          code |= C_HAS_R;
          has_r = true;
          if (!(code & C_TIR)) {
            code |= C_HAS_T;
            has_t = true;
          }
        }
      }
      q.code[i] = code;
      serve_flag(out, pix, pf);
      if (out.sig) {
        // the tracer's path signature: (generation, TIR, triangle + 1) mixed
        const bool tir = (code & C_TIR) && !(code & C_TRUNC);
        const uint64_t key = ((uint64_t)sf_depth(fl) << 40) | ((uint64_t)(tir ? 1u : 0u) << 32) |
                             (uint64_t)(uint32_t)(h.tri + 1);
        atomicAdd(out.sig + pix, (unsigned long long)path_mix64(key));
      }
    }
    uint64_t br = __ballot(has_r), bt = __ballot(has_t);
    if (lane == 0 && (br | bt))
      atomicAdd(part + base / DT_CHUNK,
                (unsigned long long)__popcll(br) | ((unsigned long long)__popcll(bt) << 32));
  }
}

// Misses of the current queue lit by environment env, listed for the MLP
// kernel: a block ranks its matches in LDS and reserves their slots with one
// atomic on ctr.nmiss[0] (zeroed before each environment's pass).
constexpr int SLB = 1024;

__global__ void __launch_bounds__(SLB) k_serve_list_env(Gen q, ServeState* st, uint32_t env,
                                                        uint32_t* list) {
  __shared__ uint32_t wcount[SLB / 64];
  __shared__ uint32_t bbase;
  Counters* ctr = &st->ctr;
  const uint32_t n = ctr->count[0];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t base = (int64_t)blockIdx.x * SLB; base < n; base += (int64_t)gridDim.x * SLB) {
    int64_t i = base + threadIdx.x;
    bool m = false;
    if (i < n && !(q.code[i] & C_HIT))
      m = sf_env((uint32_t)__float_as_int(q.w[i].w)) == env;
    uint64_t bm = __ballot(m);
    if (lane == 0) wcount[wave] = (uint32_t)__popcll(bm);
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t tot = 0;
      for (int w = 0; w < SLB / 64; ++w) {
        uint32_t c = wcount[w];
        wcount[w] = tot;
        tot += c;
      }
      bbase = tot ? atomicAdd(&ctr->nmiss[0], tot) : 0u;
    }
    __syncthreads();
    if (m) list[bbase + wcount[wave] + (uint32_t)__popcll(bm & ((1ull << lane) - 1ull))] = (uint32_t)i;
    __syncthreads();
  }
}

__global__ void k_serve_zero_nmiss(ServeState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) st->ctr.nmiss[0] = 0;
}

__global__ void __launch_bounds__(EBS) k_serve_emit(const ServeTables* T, Gen q, Gen nx,
                                                    ServeState* st, const unsigned long long* part,
                                                    int64_t cap, ServeOut out) {
  __shared__ uint32_t wr[EBS / 64], wt[EBS / 64];
  Counters* ctr = &st->ctr;
  const uint32_t n = ctr->count[0];
  const int64_t base = (int64_t)blockIdx.x * DT_CHUNK;
  if (base >= n) return;
  const uint32_t nr_tot = ctr->nrefl[0];
  unsigned long long c = part[blockIdx.x];
  uint32_t carry_r = (uint32_t)(c & 0xffffffffull), carry_t = (uint32_t)(c >> 32);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint64_t lt = (1ull << lane) - 1ull;
  for (int s = 0; s < DT_CHUNK / EBS; ++s) {
    int64_t i = base + (int64_t)s * EBS + threadIdx.x;
    bool active = i < n;
    uint32_t code = active ? q.code[i] : 0u;
    bool hr = (code & C_HAS_R) != 0u, ht = (code & C_HAS_T) != 0u;
    uint64_t br = __ballot(hr), bt = __ballot(ht);
    if (lane == 0) {
      wr[wv] = (uint32_t)__popcll(br);
      wt[wv] = (uint32_t)__popcll(bt);
    }
    __syncthreads();
    uint32_t or_ = 0, ot = 0, tr = 0, tt = 0;
    for (int k = 0; k < EBS / 64; ++k) {
      if (k < wv) {
        or_ += wr[k];
        ot += wt[k];
      }
      tr += wr[k];
      tt += wt[k];
    }
    uint32_t ir = carry_r + or_ + (uint32_t)__popcll(br & lt);
    uint32_t it = nr_tot + carry_t + ot + (uint32_t)__popcll(bt & lt);
    if (active && (hr || ht)) {
      float4 o4 = q.o[i], d4 = q.d[i], w4 = q.w[i], h4 = q.hit[i];
      v3 o = xyz(o4), d = xyz(d4), W = xyz(w4);
      int pix = __float_as_int(d4.w);
      int tri = __float_as_int(h4.y);
      uint32_t fl = (uint32_t)__float_as_int(w4.w);
      const SceneDev& sc = T->sc[sf_scene(fl)];
      HitGeo geo = load_geo(sc, tri);
      Shade sh = shade(sc, geo, o, d, h4.x, h4.z, h4.w, code);
      v3 wa = mk3(W.x * sh.A.x, W.y * sh.A.y, W.z * sh.A.z);
      bool entering = (code & C_ENTER) != 0u;
      uint32_t dep = sf_depth(fl) + 1;
      uint32_t keep = fl & ~(SF_INSIDE | (31u << 1));
      if (hr) {
        if ((int64_t)ir < cap) {
          uint32_t f2 = keep | (dep << 1) | (entering ? 0u : SF_INSIDE);
          nx.o[ir] = make_float4(sh.x.x, sh.x.y, sh.x.z, __int_as_float(tri));
          nx.d[ir] = make_float4(sh.dr.x, sh.dr.y, sh.dr.z, __int_as_float(pix));
          v3 w3 = wa * sh.R;
          nx.w[ir] = make_float4(w3.x, w3.y, w3.z, __int_as_float((int)f2));
        } else {
          serve_drop(out, &ctr->dropped, sf_slot(fl), pix);
        }
      }
      if (ht) {
        if ((int64_t)it < cap) {
          uint32_t f2 = keep | (dep << 1) | (entering ? SF_INSIDE : 0u);
          nx.o[it] = make_float4(sh.x.x, sh.x.y, sh.x.z, __int_as_float(tri));
          nx.d[it] = make_float4(sh.dt.x, sh.dt.y, sh.dt.z, __int_as_float(pix));
          v3 w3 = wa * sh.T;
          nx.w[it] = make_float4(w3.x, w3.y, w3.z, __int_as_float((int)f2));
        } else {
          serve_drop(out, &ctr->dropped, sf_slot(fl), pix);
        }
      }
    }
    carry_r += tr;
    carry_t += tt;
    __syncthreads();
  }
}

// next queue becomes current; bookkeeping for the host
__global__ void k_serve_advance(ServeState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    Counters& c = st->ctr;
    st->traced += c.count[0];
    st->dropped += c.dropped;
    c.dropped = 0;
    c.count[0] = c.count[1];
    c.count[1] = 0;
    c.nrefl[0] = 0;
    for (int x = 0; x < DT_WORK_PARTS; ++x) st->wp[x].next = 0;
  }
}

// rays per request slot in the (new) current queue
__global__ void k_slot_hist(Gen q, const ServeState* st, uint32_t* live) {
  __shared__ uint32_t h[DT_SERVE_MAX_SLOTS];
  for (int k = threadIdx.x; k < DT_SERVE_MAX_SLOTS; k += blockDim.x) h[k] = 0;
  __syncthreads();
  const uint32_t n = st->ctr.count[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&h[sf_slot((uint32_t)__float_as_int(q.w[i].w))], 1u);
  __syncthreads();
  for (int k = threadIdx.x; k < DT_SERVE_MAX_SLOTS; k += blockDim.x)
    if (h[k]) atomicAdd(&live[k], h[k]);
}

__global__ void k_serve_stats(const ServeState* st, int64_t* stats) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    stats[0] = st->traced;
    stats[1] = st->dropped;
    stats[2] = st->ctr.count[0];
  }
}

__global__ void k_zero(float* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

unsigned grid_for(int64_t n, int threads, int64_t lim) {
  int64_t b = (n + threads - 1) / threads;
  if (b > lim) b = lim;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

extern "C" dt_status dt_serve_bytes(int64_t queue_capacity, size_t* ws_bytes) {
  DT_REQUIRE(ws_bytes, "dt_serve_bytes: NULL argument");
  DT_REQUIRE(queue_capacity >= 64 && queue_capacity < (1ll << 31),
             "dt_serve_bytes: queue_capacity must be in [64, 2^31)");
  *ws_bytes = serve_layout(queue_capacity).total;
  return DT_OK;
}

extern "C" dt_status dt_serve_reset(void* ws, size_t ws_bytes, int64_t queue_capacity, void* stream) {
  DT_REQUIRE(ws, "dt_serve_reset: NULL workspace");
  DT_REQUIRE(queue_capacity >= 64 && queue_capacity < (1ll << 31), "bad queue_capacity");
  ServeLayout L = serve_layout(queue_capacity);
  if (ws_bytes < L.total) {
    dt_set_error("dt_serve_reset: workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    return DT_ERR_WORKSPACE_TOO_SMALL;
  }
  char* W = (char*)ws;
  hipLaunchKernelGGL(k_serve_reset, dim3(grid_for(L.maxchunks + 1, 256, 1024)), dim3(256), 0,
                     (hipStream_t)stream, (ServeState*)(W + L.state),
                     (unsigned long long*)(W + L.part0), (unsigned long long*)(W + L.part1),
                     L.maxchunks + 1);
  DT_CHECK_LAUNCH();
  return DT_OK;
}

extern "C" dt_status dt_serve_step(const dt_serve_scene* scenes, int32_t n_scenes, const dt_env* envs,
                                   int32_t n_envs, const dt_serve_admit* admits, int32_t n_admits,
                                   int64_t step, float* pixels, int32_t* flags, uint64_t* path_sig,
                                   int64_t n_pixels, uint32_t* slot_live, uint32_t* slot_dropped,
                                   int64_t* stats, int64_t queue_capacity, float t_eps, void* ws,
                                   size_t ws_bytes, void* stream) {
  DT_REQUIRE(scenes && envs && pixels && slot_live && slot_dropped && ws,
             "dt_serve_step: NULL argument");
  DT_REQUIRE(n_scenes >= 1 && n_scenes <= DT_SERVE_MAX_SCENES, "n_scenes must be in [1, %d]",
             DT_SERVE_MAX_SCENES);
  DT_REQUIRE(n_envs >= 1 && n_envs <= DT_SERVE_MAX_ENVS, "n_envs must be in [1, %d]",
             DT_SERVE_MAX_ENVS);
  DT_REQUIRE(n_admits >= 0 && (n_admits == 0 || admits), "bad admits");
  DT_REQUIRE(step >= 0 && n_pixels >= 1 && n_pixels < (1ll << 31), "bad step or n_pixels");
  DT_REQUIRE(t_eps >= 0.f && t_eps < 1.f, "t_eps must be in [0, 1)");
  DT_REQUIRE(queue_capacity >= 64 && queue_capacity < (1ll << 31), "bad queue_capacity");
  ServeLayout L = serve_layout(queue_capacity);
  if (ws_bytes < L.total) {
    dt_set_error("dt_serve_step: workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    return DT_ERR_WORKSPACE_TOO_SMALL;
  }
  // descriptor tables (copied into the workspace for per-ray lookup)
  ServeTables T;
  memset(&T, 0, sizeof(T));
  for (int i = 0; i < n_scenes; ++i) {
    const dt_serve_scene& s = scenes[i];
    DT_REQUIRE(s.V && s.F && s.bvh && s.ior && s.sigma && s.nv >= 3 && s.nf >= 1 &&
                   s.nf <= DT_MAX_FACES,
               "scene %d has a NULL pointer or a bad size", i);
    SceneDev& d = T.sc[i];
    d.V = s.V;
    d.F = s.F;
    d.nv = s.nv;
    d.nf = s.nf;
    d.bvh = bvh_view(s.bvh, s.nv, s.nf);
    d.ior = s.ior;
    d.sigma = s.sigma;
    d.max_depth = DT_MAX_DEPTH;
    d.terminal_env = 0;
    d.t_eps = t_eps;
  }
  for (int i = 0; i < n_envs; ++i)
    if (dt_status st = make_env(&envs[i], T.env[i])) return st;
  int64_t added = 0;
  for (int a = 0; a < n_admits; ++a) {
    const dt_serve_admit& ad = admits[a];
    DT_REQUIRE(ad.slot >= 0 && ad.slot < DT_SERVE_MAX_SLOTS, "admit %d: slot out of range", a);
    DT_REQUIRE(ad.scene >= 0 && ad.scene < n_scenes, "admit %d: scene out of range", a);
    DT_REQUIRE(ad.env >= 0 && ad.env < n_envs, "admit %d: env out of range", a);
    DT_REQUIRE(ad.max_depth >= 0 && ad.max_depth <= DT_MAX_DEPTH, "admit %d: bad max_depth", a);
    const dt_camera& c = ad.camera;
    DT_REQUIRE(c.width >= 1 && c.height >= 1 && c.fov_deg > 0.f && c.fov_deg < 180.f,
               "admit %d: bad camera", a);
    DT_REQUIRE(c.pixel_offset >= 0 && c.pixel_offset + (int64_t)c.width * c.height <= n_pixels,
               "admit %d: image exceeds the pixel pool", a);
    added += (int64_t)c.width * c.height;
  }
  hipStream_t s = (hipStream_t)stream;
  char* W = (char*)ws;
  ServeState* st = (ServeState*)(W + L.state);
  ServeTables* Td = (ServeTables*)(W + L.tables);
  hipLaunchKernelGGL(k_set_tables, dim3(1), dim3(256), 0, s, T, Td);
  ServeOut out{pixels, flags, (unsigned long long*)path_sig, slot_dropped};
  unsigned long long* part[2] = {(unsigned long long*)(W + L.part0),
                                 (unsigned long long*)(W + L.part1)};
  const int cur = (int)(step & 1), nxt = cur ^ 1;
  Gen qc = serve_gen(W, L, cur), qn = serve_gen(W, L, nxt);
  // admit: clear the requests' images, append their camera rays
  int64_t prefix = 0;
  for (int a = 0; a < n_admits; ++a) {
    const dt_serve_admit& ad = admits[a];
    CamDev cd;
    if (dt_status e = make_camera(ad.camera, a, cd)) return e;
    int64_t np = (int64_t)cd.W * cd.H;
    hipLaunchKernelGGL(k_serve_clear, dim3(grid_for(np, 256, 4096)), dim3(256), 0, s, out,
                       ad.camera.pixel_offset, np, (uint32_t)ad.slot);
    uint32_t fl = sf_make(0, 0, (uint32_t)ad.max_depth, (uint32_t)ad.scene, (uint32_t)ad.env,
                          (uint32_t)ad.slot);
    hipLaunchKernelGGL(k_serve_raygen, dim3(dt_blocks(np, 256)), dim3(256), 0, s, qc, st, prefix, cd,
                       fl, L.cap, out);
    prefix += np;
  }
  if (added) hipLaunchKernelGGL(k_serve_admit_count, dim3(1), dim3(64), 0, s, st, added, L.cap);
  DT_CHECK_LAUNCH();
  // one interaction for every live ray
  hipLaunchKernelGGL(k_serve_trace, dim3(grid_for(L.cap, TBS, SERVE_TRACE_BLOCKS)), dim3(TBS), 0, s,
                     Td, qc, st, part[cur], out, (uint2*)(W + L.ovf));
  // MLP environments: list each one's misses, evaluate them on the matrix cores
  for (int e = 0; e < n_envs; ++e) {
    if (T.env[e].kind != DT_ENV_MLP) continue;
    uint32_t* list = (uint32_t*)(W + L.miss);
    hipLaunchKernelGGL(k_serve_zero_nmiss, dim3(1), dim3(64), 0, s, st);
    hipLaunchKernelGGL(k_serve_list_env, dim3(grid_for(L.cap, SLB, 2048)), dim3(SLB), 0, s, qc, st,
                       (uint32_t)e, list);
    DT_CHECK_LAUNCH();
    if (dt_status er = mlp_trace_forward(T.env[e], qc, list, &st->ctr, 0, L.cap, pixels, s)) return er;
  }
  if (dt_status e = chunk_scan(&st->ctr, 0, part[cur], part[nxt], L.maxchunks + 1, L.cap, s)) return e;
  hipLaunchKernelGGL(k_serve_emit, dim3((unsigned)L.maxchunks), dim3(EBS), 0, s, Td, qc, qn, st,
                     part[cur], L.cap, out);
  // (the scan zeroed part[nxt] for the next step; the next step's scan zeroes part[cur])
  hipLaunchKernelGGL(k_serve_advance, dim3(1), dim3(64), 0, s, st);
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s, (float*)slot_live, (int64_t)DT_SERVE_MAX_SLOTS);
  hipLaunchKernelGGL(k_slot_hist, dim3(grid_for(L.cap, 256, 1024)), dim3(256), 0, s, qn, st, slot_live);
  if (stats) hipLaunchKernelGGL(k_serve_stats, dim3(1), dim3(64), 0, s, st, stats);
  DT_CHECK_LAUNCH();
  return DT_OK;
}
